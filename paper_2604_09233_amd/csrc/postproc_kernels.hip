// k-space filter of the reconstructed image (Methods, "Computation of
// k-space filters"; last line of both reconstruction listings):
// rho_f = IFFT(FFT(rho) o f).  It is applied with the library's own encoding
// operator: on a Cartesian grid with unit sensitivity, no B0 and linear
// phase terms only, E is the DFT, so rho_f = (1 / L) E^H diag(f) E rho with E
// the DFT of the image grid.  This kernel writes that problem.
#include "nfs_internal.h"

namespace nfs {

// voxel / sample index l = x + nx (y + ny z) for both sides
__global__ void dft_problem_kernel(int nx, int ny, int nz, float2* __restrict__ sens, float* __restrict__ fields,
                                   float* __restrict__ b0, float* __restrict__ kcoef, float* __restrict__ t) {
  const int64_t L = (int64_t)nx * ny * nz;
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  const int P = nz > 1 ? 3 : 2;
  const int ix = (int)(l % nx), iy = (int)((l / nx) % ny), iz = (int)(l / ((int64_t)nx * ny));
  const int idx[3] = {ix, iy, iz}, n[3] = {nx, ny, nz};
  sens[l] = make_float2(1.f, 0.f);
  b0[l] = 0.f;
  t[l] = 0.f;
  for (int d = 0; d < P; ++d) {
    // centred pixel index: shifts E by a sign (-1)^f per bin, which
    // E^H diag(w) E does not see, and halves the largest phase
    fields[(int64_t)d * L + l] = (float)(idx[d] - n[d] / 2);
    // signed frequency of bin idx[d] (numpy.fft.fftfreq convention)
    const int f = idx[d] < (n[d] + 1) / 2 ? idx[d] : idx[d] - n[d];
    kcoef[l * P + d] = (float)(-2.0 * 3.14159265358979323846 * (double)f / (double)n[d]);
  }
}

hipError_t launch_dft_problem(int nx, int ny, int nz, float2* sens, float* fields, float* b0, float* kcoef, float* t,
                              hipStream_t s) {
  const int64_t L = (int64_t)nx * ny * nz;
  if (L == 0) return hipSuccess;
  hipLaunchKernelGGL(dft_problem_kernel, dim3((unsigned)cdiv(L, 256)), dim3(256), 0, s, nx, ny, nz, sens, fields, b0,
                     kcoef, t);
  return hipGetLastError();
}

}  // namespace nfs
