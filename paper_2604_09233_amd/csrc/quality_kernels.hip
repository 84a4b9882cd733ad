// Stopping-criteria instrumentation: SSIM of magnitude images against a
// reference (the image-quality measure of the paper's CG-convergence
// study), on the GPU in float64.
//
// Definition (Wang, Bovik, Sheikh and Simoncelli, 2004, cited by the paper):
// Gaussian window sigma = 1.5 truncated to 11 taps per axis and normalised;
// C1 = (0.01 D)^2, C2 = (0.03 D)^2 with D = max - min of the reference
// magnitude; window-weighted mean, variance and covariance (no sample-size
// correction) at every window position fully inside the image; the result is
// the mean of the SSIM map over those positions.
//
// Layout: images are [n_img][L] complex with voxel index x + nx (y + ny z);
// the separable window runs as one pass per axis over the five moment maps
// (a, b, a^2, b^2, ab with a = |image|, b = |reference|), each pass
// shrinking its axis by 10 ("valid" filtering).  Sums are in a fixed order.
#include <cmath>

#include "nfs_internal.h"

namespace nfs {

constexpr int kSsimTaps = 11;

// the normalised window taps, computed once on the host in float64
struct SsimTaps {
  double w[kSsimTaps];
};

static SsimTaps ssim_taps() {
  SsimTaps t;
  double s = 0.0;
  for (int k = 0; k < kSsimTaps; ++k) {
    const double d = k - (kSsimTaps - 1) / 2;
    t.w[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    s += t.w[k];
  }
  for (int k = 0; k < kSsimTaps; ++k) t.w[k] /= s;
  return t;
}

// block maxima and minima of |ref| (kBmaxBlocks workgroups, every entry written)
__global__ __launch_bounds__(256) void ssim_range_kernel(const float2* __restrict__ ref, int64_t L,
                                                         double* __restrict__ part) {
  __shared__ double mx[256], mn[256];
  double hi = -INFINITY, lo = INFINITY;
  for (int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x; l < L; l += (int64_t)gridDim.x * 256) {
    const float2 v = ref[l];
    const double m = sqrt((double)v.x * v.x + (double)v.y * v.y);
    hi = fmax(hi, m);
    lo = fmin(lo, m);
  }
  mx[threadIdx.x] = hi;
  mn[threadIdx.x] = lo;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + w]);
      mn[threadIdx.x] = fmin(mn[threadIdx.x], mn[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = mx[0];
    part[kBmaxBlocks + blockIdx.x] = mn[0];
  }
}

// x pass: out[img][k][z][y][xo] = sum_dx w[dx] m_k(x = xo + dx), with the
// moments m_k formed from the complex inputs
__global__ __launch_bounds__(256) void ssim_pass_x_kernel(const float2* __restrict__ imgs, const float2* __restrict__ ref,
                                                          int n_img, int nx, int ny, int nz, SsimTaps tw,
                                                          double* __restrict__ out) {
  const int nxo = nx - (kSsimTaps - 1);
  const int64_t L = (int64_t)nx * ny * nz;
  const int64_t per_img = (int64_t)nz * ny * nxo;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= per_img * n_img) return;
  const int img = (int)(i / per_img);
  const int64_t r = i - img * per_img;
  const int xo = (int)(r % nxo);
  const int64_t row = r / nxo;  // z * ny + y
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int dx = 0; dx < kSsimTaps; ++dx) {
    const int64_t l = row * nx + xo + dx;
    const float2 u = imgs[(int64_t)img * L + l], v = ref[l];
    const double a = sqrt((double)u.x * u.x + (double)u.y * u.y);
    const double b = sqrt((double)v.x * v.x + (double)v.y * v.y);
    const double w = tw.w[dx];
    s[0] += w * a;
    s[1] += w * b;
    s[2] += w * a * a;
    s[3] += w * b * b;
    s[4] += w * a * b;
  }
  for (int k = 0; k < 5; ++k) out[((int64_t)img * 5 + k) * per_img + r] = s[k];
}

// pass along an axis of stride `stride` (y: nxo, z: nyo * nxo) over arrays
// [img][5][outer][axis][inner]: out axis length n_out = n_in - 10
__global__ __launch_bounds__(256) void ssim_pass_kernel(const double* __restrict__ in, int n_img, int64_t outer,
                                                        int n_in, int64_t inner, SsimTaps tw, double* __restrict__ out) {
  const int n_out = n_in - (kSsimTaps - 1);
  const int64_t per_in = outer * n_in * inner, per_out = outer * n_out * inner;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= per_out * 5 * n_img) return;
  const int64_t ik = i / per_out;  // img * 5 + k
  const int64_t r = i - ik * per_out;
  const int64_t in_ = r % inner;
  const int64_t t = r / inner;
  const int ao = (int)(t % n_out);
  const int64_t o = t / n_out;
  const double* src = in + ik * per_in + (o * n_in + ao) * inner + in_;
  double s = 0.0;
  for (int d = 0; d < kSsimTaps; ++d) s += tw.w[d] * src[(int64_t)d * inner];
  out[i] = s;
}

// SSIM map and its mean per image: one workgroup per image, fixed-order
// tree; D from the range partials (summed in the same order everywhere)
__global__ __launch_bounds__(256) void ssim_mean_kernel(const double* __restrict__ mom, int64_t npos,
                                                        const double* __restrict__ range_part,
                                                        double* __restrict__ out) {
  __shared__ double red[256];
  const int img = blockIdx.x;
  double hi = -INFINITY, lo = INFINITY;
  for (int b = 0; b < kBmaxBlocks; ++b) {
    hi = fmax(hi, range_part[b]);
    lo = fmin(lo, range_part[kBmaxBlocks + b]);
  }
  const double D = hi - lo;
  const double c1 = (0.01 * D) * (0.01 * D), c2 = (0.03 * D) * (0.03 * D);
  const double* m = mom + (int64_t)img * 5 * npos;
  double acc = 0.0;
  for (int64_t p = threadIdx.x; p < npos; p += 256) {
    const double ma = m[p], mb = m[npos + p];
    const double va = m[2 * npos + p] - ma * ma, vb = m[3 * npos + p] - mb * mb;
    const double cv = m[4 * npos + p] - ma * mb;
    acc += ((2 * ma * mb + c1) * (2 * cv + c2)) / ((ma * ma + mb * mb + c1) * (va + vb + c2));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[img] = red[0] / (double)npos;
}

static inline dim3 grid256(int64_t n) { return dim3((unsigned)cdiv(n, 256)); }

size_t ssim_workspace_bytes(int n_img, int nx, int ny, int nz) {
  const int64_t nxo = nx - 10;
  const size_t a = (size_t)n_img * 5 * (size_t)nz * ny * nxo * 8;  // after the x pass (also after z)
  const size_t b = (size_t)n_img * 5 * (size_t)nz * (ny - 10) * nxo * 8;  // after the y pass
  return ((a + 255) & ~(size_t)255) + ((b + 255) & ~(size_t)255) + 2 * kBmaxBlocks * 8;
}

hipError_t launch_ssim(const float2* imgs, int n_img, const float2* ref, int nx, int ny, int nz, double* out, void* ws,
                       hipStream_t s) {
  if (n_img == 0) return hipSuccess;
  const int64_t L = (int64_t)nx * ny * nz;
  const int nxo = nx - 10, nyo = ny - 10, nzo = nz > 1 ? nz - 10 : 1;
  const size_t a = (size_t)n_img * 5 * (size_t)nz * ny * nxo * 8;
  double* bufA = static_cast<double*>(ws);
  double* bufB = reinterpret_cast<double*>(static_cast<char*>(ws) + ((a + 255) & ~(size_t)255));
  const size_t b = (size_t)n_img * 5 * (size_t)nz * nyo * nxo * 8;
  double* range = reinterpret_cast<double*>(reinterpret_cast<char*>(bufB) + ((b + 255) & ~(size_t)255));
  hipLaunchKernelGGL(ssim_range_kernel, dim3(kBmaxBlocks), dim3(256), 0, s, ref, L, range);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const SsimTaps tw = ssim_taps();
  hipLaunchKernelGGL(ssim_pass_x_kernel, grid256((int64_t)n_img * nz * ny * nxo), dim3(256), 0, s, imgs, ref, n_img,
                     nx, ny, nz, tw, bufA);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // y pass: [img][5][z][y][xo] -> [img][5][z][yo][xo]
  hipLaunchKernelGGL(ssim_pass_kernel, grid256((int64_t)n_img * 5 * nz * nyo * nxo), dim3(256), 0, s, bufA, n_img,
                     (int64_t)nz, ny, (int64_t)nxo, tw, bufB);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const double* mom = bufB;
  if (nz > 1) {
    // z pass: [img][5][z][yo*xo] -> [img][5][zo][yo*xo]
    hipLaunchKernelGGL(ssim_pass_kernel, grid256((int64_t)n_img * 5 * nzo * nyo * nxo), dim3(256), 0, s, bufB, n_img,
                       (int64_t)1, nz, (int64_t)nyo * nxo, tw, bufA);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    mom = bufA;
  }
  hipLaunchKernelGGL(ssim_mean_kernel, dim3(n_img), dim3(256), 0, s, mom, (int64_t)nzo * nyo * nxo, range, out);
  return hipGetLastError();
}

}  // namespace nfs
