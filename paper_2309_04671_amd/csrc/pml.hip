// Damping profile of the absorbing layer ("PML" region of the paper's
// Sec. 2.2).  The layer update itself is the MODE_PML sweep of k_star25
// (star25.hip), launched on the layer's boxes by sp_wave_step_pml.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace sp {

namespace {

__global__ void k_pml_profile(float *eta, int64_t sy, int64_t sz, int nx, int ny, int nz, int w,
                              float eta_max) {
    const int px = nx + 8, py = ny + 8, pz = nz + 8;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)px * py * pz) return;
    const int x = (int)(t % px) - 4;
    const int y = (int)((t / px) % py) - 4;
    const int z = (int)(t / ((int64_t)px * py)) - 4;
    auto depth = [&](int q, int n) { return (float)max(0, max(w - 1 - q, q - (n - w))) / (float)w; };
    const float dx = depth(x, nx), dy = depth(y, ny), dz = depth(z, nz);
    eta[(int64_t)z * sz + (int64_t)y * sy + x] = eta_max * (dz * dz + dy * dy + dx * dx);
}

}  // namespace

hipError_t launch_pml_profile(float *eta, int64_t sy, int64_t sz, int nx, int ny, int nz, int width,
                              float eta_max, hipStream_t s) {
    const int64_t n = (int64_t)(nx + 8) * (ny + 8) * (nz + 8);
    const int bs = 256;
    hipLaunchKernelGGL(k_pml_profile, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, eta, sy, sz,
                       nx, ny, nz, width, eta_max);
    return hipGetLastError();
}

}  // namespace sp
