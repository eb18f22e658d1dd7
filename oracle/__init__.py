"""Oracle: a plain, slow, CPU reference of the directional-distance-field hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: it is used by ``tests/``, by the smoke check in
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``.  It shares no
code with the HIP path; both read the same seeded inputs from ``synthetic``.

Everything is computed in float64 with NumPy (matrix products through NumPy's
matmul) unless a function states an emulated reduced precision.  Each function
cites the passage of the paper (arXiv 2306.16142) it follows.

Modules:
* ``geometry`` -- direction <-> angle parametrisation (Sec. III-A, Eq. 1),
  cube entry, brute-force nearest ray/triangle hit (Sec. I linear search,
  Sec. V-B odd-even rule), Moller-Trumbore form.
* ``mlp``      -- Fourier encoding, network forward in float64 and with emulated
  bfloat16 / fp8-e4m3 operands, loss seeds, backward (Sec. IV-B gradient with
  respect to the input point), Adam, normals (Eq. 3).
* ``render``   -- counter-based random numbers (SplitMix64) and the path tracer
  of Fig. 1 with a mesh or a network backend.
* ``dataset``  -- the informative training-data sampler of Sec. V-B
  (Eqs. 8-12): face points, direction samples, marching, infinite samples.
* ``udf``      -- the unsigned distance field as the minimum of the field over
  a direction set (Sec. III-A, Eq. 5).
* ``multi``    -- rigid instances of several networks (Sec. VII, scenes as
  future work).

Parity status of every function is listed in its docstring ("pinned by ...").
"""
