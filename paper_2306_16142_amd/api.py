"""Thin PyTorch binding of libddf: allocates outputs as torch CUDA tensors and passes
raw device pointers and the current HIP stream to the C ABI.  Every step of the hot
path runs in the library's kernels; nothing here computes."""
import ctypes
import math

import torch

from . import _lib

PRECISIONS = {"fp32": _lib.PREC_FP32, "bf16": _lib.PREC_BF16, "fp8": _lib.PREC_FP8}


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name, rows=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if rows is not None and (t.dim() != 2 or t.shape[0] != rows):
        raise ValueError("%s must have shape [%d, n], got %s" % (name, rows, tuple(t.shape)))
    return t


def label_rays(orig, dirs, tris, t_min=0.0, t_max=math.inf, crossings=True):
    """Nearest triangle hit of every ray: returns (t [n], tri [n] int32, crossings [n] int32 or None)."""
    _dev(orig, torch.float32, "orig", 3)
    _dev(dirs, torch.float32, "dirs", 3)
    _dev(tris, torch.float32, "tris", 9)
    n, m = orig.shape[1], tris.shape[1]
    t = torch.empty(n, device=orig.device, dtype=torch.float32)
    tri = torch.empty(n, device=orig.device, dtype=torch.int32)
    cr = torch.empty(n, device=orig.device, dtype=torch.int32) if crossings else None
    _lib.call("ddf_label_rays", _p(orig), _p(dirs), n, _p(tris), m, t_min, t_max, _p(t), _p(tri), _p(cr), _stream())
    return t, tri, cr


def assemble_rays(orig, dirs, out=None):
    """(origins [3][n], directions [3][n]) -> rays [5][n] = (ox, oy, oz, theta, phi)."""
    _dev(orig, torch.float32, "orig", 3)
    _dev(dirs, torch.float32, "dirs", 3)
    n = orig.shape[1]
    out = torch.empty((5, n), device=orig.device, dtype=torch.float32) if out is None else out
    _lib.call("ddf_assemble_rays", _p(orig), _p(dirs), n, _p(out), _stream())
    return out


def udf_workspace_bytes(n_points, n_dirs):
    b = ctypes.c_size_t(0)
    _lib.call("ddf_udf_workspace_size", n_points, n_dirs, ctypes.byref(b))
    return b.value


def udf(net, points, dirs, out=None, arg=None, workspace=None):
    """Unsigned distance field (Eq. 5): the minimum over the unit directions ``dirs`` [3][d]
    of the network's distance from each of ``points`` [3][n] (misses: +inf).  Returns
    (udf [n], argmin direction [n] int32, -1 where every direction misses)."""
    _dev(points, torch.float32, "points", 3)
    _dev(dirs, torch.float32, "dirs", 3)
    n, d = points.shape[1], dirs.shape[1]
    out = torch.empty(n, device=points.device, dtype=torch.float32) if out is None else out
    arg = torch.empty(n, device=points.device, dtype=torch.int32) if arg is None else arg
    if workspace is None:
        workspace = torch.empty(max(udf_workspace_bytes(n, d), 1), device=points.device, dtype=torch.uint8)
    _lib.call("ddf_udf", ctypes.byref(net.desc), _p(points), n, _p(dirs), d, _p(out), _p(arg), _p(workspace),
              workspace.numel(), _stream())
    return out, arg


class DatasetSampler:
    """The training-data sampler of Sec. V-B (``ddf_sample_dataset``) with its workspace and
    output buffers allocated once (capacity: every possible sample, 4 per marching step)."""

    def __init__(self, tris, s_fc, s_dr, s_p, eps=1e-4, face_first=0, n_faces=None, device="cuda"):
        _dev(tris, torch.float32, "tris", 9)
        self.tris, self.m = tris, tris.shape[1]
        n_faces = self.m - face_first if n_faces is None else n_faces
        self.params = _lib.DdfDatasetParams(s_fc, s_dr, s_p, eps, face_first, n_faces)
        b = ctypes.c_size_t(0)
        _lib.call("ddf_dataset_workspace_size", ctypes.byref(self.params), ctypes.byref(b))
        self.ws = torch.empty(max(b.value, 1), device=tris.device, dtype=torch.uint8)
        self.cap = 4 * n_faces * s_fc * s_dr * s_p
        self.rays = torch.empty((5, self.cap), device=tris.device, dtype=torch.float32)
        self.t = torch.empty(self.cap, device=tris.device, dtype=torch.float32)
        self.pair = torch.empty(self.cap, device=tris.device, dtype=torch.int32)
        self.count = torch.zeros(1, device=tris.device, dtype=torch.int64)

    def run(self, face_uv, dir_uv, pairs=True):
        """Enqueue one sampling pass; the sample count lands in ``self.count`` (device)."""
        _dev(face_uv, torch.float32, "face_uv", 2)
        _dev(dir_uv, torch.float32, "dir_uv", 2)
        _lib.call("ddf_sample_dataset", _p(self.tris), self.m, ctypes.byref(self.params), _p(face_uv), _p(dir_uv),
                  _p(self.rays), _p(self.t), _p(self.pair) if pairs else None, self.cap, _p(self.count),
                  _p(self.ws), self.ws.numel(), _stream())

    def __call__(self, face_uv, dir_uv):
        """Sample and return (rays [5][N], t [N], pair [N]) views of the output buffers."""
        self.run(face_uv, dir_uv)
        n = int(self.count.item())
        return self.rays[:, :n], self.t[:n], self.pair[:n]


def packed_bytes(width, depth, precision):
    b = ctypes.c_size_t(0)
    _lib.call("ddf_packed_bytes", width, depth, PRECISIONS[precision], ctypes.byref(b))
    return b.value


class Network:
    """A packed network (weights in MFMA-tile order) for one precision.

    ``params``: flat float32 CUDA tensor (per layer weight [out][in] then bias).
    For ``precision='fp8'`` give ``scales`` ([2 (depth + 1)] CUDA float32), e.g. from
    :func:`fp8_scales`.
    """

    def __init__(self, params, width, depth, precision="bf16", scales=None):
        _dev(params, torch.float32, "params")
        self.params, self.width, self.depth, self.precision = params, width, depth, precision
        self.scales = scales
        nbytes = packed_bytes(width, depth, precision)
        self.blob = torch.empty(nbytes, device=params.device, dtype=torch.uint8)
        _lib.call("ddf_pack_net", _p(params), width, depth, PRECISIONS[precision],
                  _p(scales) if scales is not None else ctypes.c_void_p(0), _p(self.blob), _stream())
        self.desc = _lib.DdfNet(width, depth, PRECISIONS[precision], self.blob.data_ptr())

    def forward(self, rays, logit=None, dist=None):
        """rays [5][n] -> (logit [n], dist [n])."""
        _dev(rays, torch.float32, "rays", 5)
        n = rays.shape[1]
        logit = torch.empty(n, device=rays.device, dtype=torch.float32) if logit is None else logit
        dist = torch.empty(n, device=rays.device, dtype=torch.float32) if dist is None else dist
        _lib.call("ddf_forward", ctypes.byref(self.desc), _p(rays), n, _p(logit), _p(dist), _stream())
        return logit, dist

    __call__ = forward

    def query(self, orig, dirs, logit=None, dist=None):
        """origins [3][n] + unit directions [3][n] -> (logit [n], dist [n]) in one kernel
        (bf16 / fp8 networks held in LDS; equal to assemble_rays + forward)."""
        _dev(orig, torch.float32, "orig", 3)
        _dev(dirs, torch.float32, "dirs", 3)
        n = orig.shape[1]
        if dirs.shape[1] != n:
            raise ValueError("orig and dirs differ in length")
        logit = torch.empty(n, device=orig.device, dtype=torch.float32) if logit is None else logit
        dist = torch.empty(n, device=orig.device, dtype=torch.float32) if dist is None else dist
        _lib.call("ddf_query", ctypes.byref(self.desc), _p(orig), _p(dirs), n, _p(logit), _p(dist), _stream())
        return logit, dist


def paper_param_count(depth):
    c = ctypes.c_int64(0)
    _lib.call("ddf_paper_param_count", depth, ctypes.byref(c))
    return c.value


def paper_workspace_bytes(depth, n):
    b = ctypes.c_size_t(0)
    _lib.call("ddf_paper_workspace_size", depth, n, ctypes.byref(b))
    return b.value


class PaperNetwork:
    """The paper's own network (Sec. V-A): ``depth`` weight-normalised hidden ReLU layers of 512
    units on the raw ray (ox, oy, oz, theta, phi), one distance output.

    ``params``: flat float32 CUDA tensor (per hidden layer v [512][in], g [512], b [512], then
    the output row [512] and bias); the weight normalisation is folded when packing.
    ``precision``: "fp32" or "bf16"."""

    def __init__(self, params, depth, precision="bf16"):
        _dev(params, torch.float32, "params")
        if params.numel() != paper_param_count(depth):
            raise ValueError("params has %d values, a depth-%d paper network needs %d"
                             % (params.numel(), depth, paper_param_count(depth)))
        self.params, self.depth, self.precision = params, depth, precision
        b = ctypes.c_size_t(0)
        _lib.call("ddf_paper_packed_bytes", depth, PRECISIONS[precision], ctypes.byref(b))
        self.blob = torch.empty(b.value, device=params.device, dtype=torch.uint8)
        self.desc = _lib.DdfPaperNet(depth, PRECISIONS[precision], self.blob.data_ptr())
        self.repack()

    def repack(self):
        _lib.call("ddf_paper_pack", _p(self.params), self.depth, PRECISIONS[self.precision], _p(self.blob), _stream())

    def forward(self, rays, dist=None):
        """rays [5][n] -> dist [n]."""
        _dev(rays, torch.float32, "rays", 5)
        n = rays.shape[1]
        dist = torch.empty(n, device=rays.device, dtype=torch.float32) if dist is None else dist
        _lib.call("ddf_paper_forward", ctypes.byref(self.desc), _p(rays), n, _p(dist), _stream())
        return dist

    __call__ = forward

    def backward(self, rays, g_dist, want_rays=True, want_params=False, g_params=None, accumulate=False,
                 workspace=None):
        """Reverse mode of sum(g_dist * dist): returns (g_rays [5][n] or None, g_params or None)."""
        _dev(rays, torch.float32, "rays", 5)
        n = rays.shape[1]
        g_rays = torch.empty((5, n), device=rays.device, dtype=torch.float32) if want_rays else None
        ws = None
        if want_params:
            if g_params is None:
                g_params = torch.zeros(self.params.numel(), device=rays.device, dtype=torch.float32)
            nb = paper_workspace_bytes(self.depth, n)
            ws = workspace if workspace is not None and workspace.numel() >= nb else \
                torch.empty(nb, device=rays.device, dtype=torch.uint8)
        else:
            g_params = None
        _lib.call("ddf_paper_backward", ctypes.byref(self.desc), _p(self.params), _p(rays), n, _p(g_dist), _p(g_rays),
                  _p(g_params),
                  1 if accumulate else 0, _p(ws), ws.numel() if ws is not None else 0, _stream())
        return g_rays, g_params


class PaperTrainer:
    """Adam training of the paper's network (float32) on labelled rays with the clamp loss
    (Eq. 7, window ``delta``) or the squish loss (Eq. 6) and dropout ``dropout`` after every
    hidden ReLU (the paper: 0.5; masks drawn from ``seed`` and the step count); ``params`` is
    updated in place."""

    def __init__(self, params, depth, batch, lr=1e-3, loss="clamp", delta=1.0, dropout=0.5, seed=0):
        self.net = PaperNetwork(params, depth, "fp32")
        self.params = params
        self.dropout = float(dropout)
        self.seed = int(seed)
        self.loss_desc = _loss_desc(loss, delta)
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.g = torch.zeros_like(params)
        self.loss = torch.zeros(1, device=params.device, dtype=torch.float32)
        self.lr = lr
        self.step_count = 0
        self.ws = torch.empty(paper_workspace_bytes(depth, batch), device=params.device, dtype=torch.uint8)

    def step(self, rays, t_label):
        _dev(rays, torch.float32, "rays", 5)
        _dev(t_label, torch.float32, "t_label")
        self.step_count += 1
        _lib.call("ddf_paper_train_step", ctypes.byref(self.net.desc), _p(self.params), _p(self.m), _p(self.v),
                  self.step_count, self.lr, _p(rays), _p(t_label), rays.shape[1], ctypes.byref(self.loss_desc),
                  self.dropout, self.seed, _p(self.loss), _p(self.g), _p(self.ws), self.ws.numel(), _stream())
        return self.loss


def train_workspace_bytes(width, depth, n):
    b = ctypes.c_size_t(0)
    _lib.call("ddf_train_workspace_size", width, depth, n, ctypes.byref(b))
    return b.value


def backward(net, rays, g_logit=None, g_dist=None, want_rays=True, want_params=False, g_params=None,
             accumulate=False, workspace=None):
    """Reverse-mode gradient of sum(g_logit * logit + g_dist * dist): returns (g_rays, g_params)."""
    _dev(rays, torch.float32, "rays", 5)
    n = rays.shape[1]
    g_rays = torch.empty((5, n), device=rays.device, dtype=torch.float32) if want_rays else None
    ws = None
    if want_params:
        if g_params is None:
            g_params = torch.zeros(net.params.numel(), device=rays.device, dtype=torch.float32)
        nb = train_workspace_bytes(net.width, net.depth, n)
        ws = workspace if workspace is not None and workspace.numel() >= nb else \
            torch.empty(nb, device=rays.device, dtype=torch.uint8)
    else:
        g_params = None
    _lib.call("ddf_backward", ctypes.byref(net.desc), _p(rays), n, _p(g_logit), _p(g_dist), _p(g_rays),
              _p(g_params), 1 if accumulate else 0, _p(ws), ws.numel() if ws is not None else 0, _stream())
    return g_rays, g_params


def _loss_desc(loss, delta):
    return _lib.DdfLoss(_lib.LOSSES[loss], delta)


def loss_seeds(logit, dist, t_label, loss="bce_l1", delta=1.0):
    """A training loss and its seeds: returns (loss [1], g_logit, g_dist).  ``loss``: "bce_l1"
    (BCE on the hit + L1 on hit distances), "clamp" (Eq. 7, window ``delta``) or "squish"
    (Eq. 6 with tanh)."""
    n = logit.numel()
    g_logit, g_dist = torch.empty_like(logit), torch.empty_like(dist)
    out = torch.empty(1, device=logit.device, dtype=torch.float32)
    ws = torch.empty(4160, device=logit.device, dtype=torch.uint8)
    desc = _loss_desc(loss, delta)
    _lib.call("ddf_loss_seeds_ex", _p(logit), _p(dist), _p(t_label), n, ctypes.byref(desc), _p(g_logit), _p(g_dist),
              _p(out), _p(ws), ws.numel(), _stream())
    return out, g_logit, g_dist


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _lib.call("ddf_adam_step", _p(params), _p(grads), _p(m), _p(v), params.numel(), step, lr, beta1, beta2, eps,
              _stream())


class Trainer:
    """Adam training of a float32 network on labelled rays (loss: BCE on hit + L1 on distance).

    The packed network ``net`` is rewritten after every step; ``params`` is updated in place.
    """

    def __init__(self, params, width, depth, batch, lr=1e-3, chunk=None, loss="bce_l1", delta=1.0):
        """``chunk``: sweep batches in column ranges of this many rays (workspace sized for
        ``chunk`` instead of ``batch``; the forward pass is recomputed per chunk).  ``loss``:
        "bce_l1" (default), "clamp" (Eq. 7, window ``delta``) or "squish" (Eq. 6, tanh)."""
        self.chunk = chunk
        self.loss_desc = _loss_desc(loss, delta)
        self.net = Network(params, width, depth, "fp32")
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.g = torch.zeros_like(params)
        self.loss = torch.zeros(1, device=params.device, dtype=torch.float32)
        self.lr = lr
        self.step_count = 0
        self.ws = torch.empty(train_workspace_bytes(width, depth, chunk if chunk else batch), device=params.device,
                              dtype=torch.uint8)

    def step(self, rays, t_label):
        _dev(rays, torch.float32, "rays", 5)
        _dev(t_label, torch.float32, "t_label")
        self.step_count += 1
        n = rays.shape[1]
        _lib.call("ddf_train_step_ex", ctypes.byref(self.net.desc), _p(self.params), _p(self.m), _p(self.v),
                  self.step_count, self.lr, _p(rays), _p(t_label), n, self.chunk or 0, ctypes.byref(self.loss_desc),
                  _p(self.loss), _p(self.g), _p(self.ws), self.ws.numel(), _stream())
        return self.loss


    def step_eikonal(self, orig, dirs, t_label, h=0.02, lam=0.1):
        """One step with the directed Eikonal penalty of Eq. 2 added (forward difference along
        each ray with step ``h``, weight ``lam``): rays given as origins + directions.  The
        doubled batch is swept whole: a Trainer built with ``chunk`` refuses this step."""
        if self.chunk:
            raise ValueError("the Eikonal step sweeps the doubled batch whole; it has no chunked form "
                             "(build the Trainer without chunk)")
        _dev(orig, torch.float32, "orig", 3)
        _dev(dirs, torch.float32, "dirs", 3)
        _dev(t_label, torch.float32, "t_label")
        n = orig.shape[1]
        b = ctypes.c_size_t(0)
        _lib.call("ddf_eikonal_workspace_size", self.net.width, self.net.depth, n, ctypes.byref(b))
        if getattr(self, "eik_ws", None) is None or self.eik_ws.numel() < b.value:
            self.eik_ws = torch.empty(b.value, device=orig.device, dtype=torch.uint8)
        self.step_count += 1
        _lib.call("ddf_train_step_eikonal", ctypes.byref(self.net.desc), _p(self.params), _p(self.m), _p(self.v),
                  self.step_count, self.lr, _p(orig), _p(dirs), _p(t_label), n, h, lam, ctypes.byref(self.loss_desc),
                  _p(self.loss), _p(self.g), _p(self.eik_ws), self.eik_ws.numel(), _stream())
        return self.loss


class DDFQuery(torch.autograd.Function):
    """torch.autograd wrapper: forward = ddf_forward, backward = ddf_backward (float32 network)."""

    @staticmethod
    def forward(ctx, rays, params, net):
        ctx.net = net
        ctx.save_for_backward(rays)
        logit, dist = net.forward(rays.contiguous())
        return logit, dist

    @staticmethod
    def backward(ctx, g_logit, g_dist):
        (rays,) = ctx.saved_tensors
        net = ctx.net
        want_params = ctx.needs_input_grad[1]
        g_rays, g_params = backward(net, rays.contiguous(), g_logit.contiguous(), g_dist.contiguous(),
                                    want_rays=ctx.needs_input_grad[0], want_params=want_params)
        return g_rays, g_params, None


def render_params(cfg, spp_chunk=0):
    """ddf_render_params from a scene description (camera / light / sizes)."""
    c = _lib.DdfRenderParams()
    c.width, c.height, c.spp, c.bounces, c.rr_start = cfg.width, cfg.height, cfg.spp, cfg.bounces, cfg.rr_start
    c.seed, c.eps = cfg.seed, cfg.eps
    c.eye[:] = list(cfg.camera.eye)
    c.target[:] = list(cfg.camera.target)
    c.up[:] = list(cfg.camera.up)
    c.vfov_deg = cfg.camera.vfov_deg
    c.light_pos[:] = list(cfg.light.position)
    c.light_intensity[:] = list(cfg.light.intensity)
    c.albedo[:] = list(cfg.albedo)
    c.spp_chunk = spp_chunk
    return c


class Renderer:
    """Wavefront path tracer.  The scene is the mesh (``tris`` [9][m]), one network (``net``),
    or several networks placed as rigid instances (``nets`` + ``instances``: dicts with ``R``
    (3x3 object to world), ``T`` (3) and ``net`` (index into ``nets``))."""

    def __init__(self, cfg, tris=None, net=None, nets=None, instances=None, spp_chunk=0, device="cuda"):
        given = [tris is not None, net is not None, nets is not None]
        if sum(given) != 1:
            raise ValueError("give exactly one of tris, net, or nets + instances")
        self.cfg = cfg
        self.params = render_params(cfg, spp_chunk)
        self.keep = (tris, net, nets)
        if net is not None:
            self.scene = _lib.DdfScene(_lib.BACKEND_NET, None, 0, ctypes.pointer(net.desc), 0, None, 0, None)
        elif tris is not None:
            _dev(tris, torch.float32, "tris", 9)
            self.scene = _lib.DdfScene(_lib.BACKEND_MESH, tris.data_ptr(), tris.shape[1], None, 0, None, 0, None)
        else:
            self.net_array = (_lib.DdfNet * len(nets))(*[n.desc for n in nets])
            inst = []
            for d in instances:
                R = [float(x) for x in list(d["R"][0]) + list(d["R"][1]) + list(d["R"][2])]
                inst.append(_lib.DdfInstance((ctypes.c_float * 9)(*R), (ctypes.c_float * 3)(*[float(x) for x in d["T"]]),
                                             int(d["net"])))
            self.inst_array = (_lib.DdfInstance * len(inst))(*inst)
            self.scene = _lib.DdfScene(_lib.BACKEND_MULTI, None, 0, None, len(nets), self.net_array, len(inst),
                                       self.inst_array)
        b = ctypes.c_size_t(0)
        _lib.call("ddf_render_workspace_size", ctypes.byref(self.scene), ctypes.byref(self.params), ctypes.byref(b))
        self.ws = torch.empty(b.value, device=device, dtype=torch.uint8)
        H, W = cfg.height, cfg.width
        self.radiance = torch.empty((3, H, W), device=device, dtype=torch.float32)
        self.depth = torch.empty((H, W), device=device, dtype=torch.float32)
        self.normal = torch.empty((3, H, W), device=device, dtype=torch.float32)
        nstats = cfg.bounces * (2 + len(nets) if nets is not None else 4)
        self.stats = torch.empty(nstats, device=device, dtype=torch.int32)

    def render(self):
        _lib.call("ddf_render_wavefront", ctypes.byref(self.scene), ctypes.byref(self.params), _p(self.radiance),
                  _p(self.depth), _p(self.normal), _p(self.stats), _p(self.ws), self.ws.numel(), _stream())
        return self.radiance

    def capture(self):
        """Records one render() into a HIP graph; replay() re-runs it.  The call makes no host
        synchronisation (every queue count lives in device memory) and clears its outputs with
        kernels, so the whole frame is capturable.  One eager render runs first so that
        one-time launch setup stays outside the capture."""
        self.render()
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.render()
        torch.cuda.synchronize()
        return self.graph

    def replay(self):
        self.graph.replay()
        return self.radiance

    def path_stats(self):
        """Per bounce: paths entering it, shadow rays traced, hits and rays of the nearest-hit
        pass (mesh and single-network scenes; a network scene queries only the rays that enter
        the cube [-1, 1]^3), pairs per network (multi-object scenes); None where a scene has
        no such count."""
        st = self.stats.cpu().numpy()
        b = self.cfg.bounces
        paths, shadows = st[:b], st[b:2 * b]
        if self.keep[2] is not None:   # multi-object
            return paths, shadows, None, None, st[2 * b:].reshape(b, -1)
        return paths, shadows, st[2 * b:3 * b], st[3 * b:4 * b], None


def fp8_scales(params, width, depth, calib_rays, net_fp32=None):
    """Static per-layer fp8 scales: powers of two covering the weight absmax and the input absmax over the calibration rays."""
    _dev(calib_rays, torch.float32, "calib_rays", 5)
    net_fp32 = net_fp32 or Network(params, width, depth, "fp32")
    out = torch.empty(2 * (depth + 1), device=params.device, dtype=torch.float32)
    _lib.call("ddf_fp8_scales", ctypes.byref(net_fp32.desc), _p(params), _p(calib_rays), calib_rays.shape[1],
              _p(out), _stream())
    return out


def set_tuning(name, value):
    """Set a launch-shape knob (``_lib.TUNE_KNOBS``); results do not change, only speed."""
    _lib.call("ddf_set_tuning", _lib.TUNE_KNOBS[name], int(value))


def get_tuning(name):
    v = ctypes.c_int32(0)
    _lib.call("ddf_get_tuning", _lib.TUNE_KNOBS[name], ctypes.byref(v))
    return v.value
