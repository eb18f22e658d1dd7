// Ray assembly: origins and direction vectors -> the 5-value oriented points (x, theta)
// the network takes (Eq. 1 read backwards: theta = polar angle from +z, phi = azimuth).
#include <cmath>

#include "common.hpp"
#include "rays_device.hpp"

namespace ddf {
namespace {

__global__ void assemble_kernel(const float *__restrict__ orig, const float *__restrict__ dir, int64_t n,
                                float *__restrict__ rays) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float theta, phi;
        dir_angles(dir[i], dir[n + i], dir[2 * n + i], theta, phi);
        rays[i] = orig[i];
        rays[n + i] = orig[n + i];
        rays[2 * n + i] = orig[2 * n + i];
        rays[3 * n + i] = theta;
        rays[4 * n + i] = phi;
    }
}

}  // namespace
}  // namespace ddf

extern "C" ddf_status ddf_assemble_rays(const float *orig, const float *dir, int64_t n, float *rays_out,
                                        ddf_stream stream) {
    using namespace ddf;
    DDF_REQUIRE(n >= 0, DDF_ERR_INVALID_ARG, "ddf_assemble_rays: negative n");
    if (n == 0) return DDF_OK;
    DDF_REQUIRE(orig && dir && rays_out, DDF_ERR_INVALID_ARG, "ddf_assemble_rays: NULL array");
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), orig, dir, n, rays_out);
    return launch_status("ddf_assemble_rays");
}
