// Direction -> angles of the network input (Eq. 1 read backwards): theta = polar angle from
// +z in [0, pi], phi = azimuth atan2(dy, dx) wrapped into [0, 2 pi).  One definition for
// every kernel that assembles rays, so they agree bit for bit.
#pragma once
#include <cmath>

namespace ddf {

constexpr float kTwoPiF = 6.28318530717958647692f;
constexpr float kBelowTwoPiF = 6.28318500518798828125f;   // largest float32 below fl(2 pi)

// The two atan2 arguments of each angle, and the wrap of the azimuth, written once (explicit
// fma) so that every caller computes the same bits.
__device__ inline float polar_y(float dx, float dy) { return sqrtf(fmaf(dx, dx, dy * dy)); }
__device__ inline float wrap_azimuth(float phi) {
    if (phi < 0.f) phi += kTwoPiF;
    if (phi >= kTwoPiF) phi = kBelowTwoPiF;
    return phi;
}

__device__ inline void dir_angles(float dx, float dy, float dz, float &theta, float &phi) {
    theta = atan2f(polar_y(dx, dy), dz);
    phi = wrap_azimuth(atan2f(dy, dx));
}

}  // namespace ddf
