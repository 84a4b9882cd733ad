// k-space filter of the reconstructed image (Methods, "Computation of
// k-space filters"; last line of both reconstruction listings):
// rho_f = IFFT(FFT(rho) o f).  The multidimensional DFT is separable, so it
// is applied one axis at a time: a pass along an axis of length n maps every
// line of the grid along that axis through the n-point DFT, n complex
// multiply-adds per output.  Forward passes over all axes, the filter (and
// 1/L) with the last forward pass, then the inverse passes.  L (nx + ny + nz)
// multiply-adds per direction instead of the L^2 of the grid's full DFT
// matrix.
#include "nfs_internal.h"

namespace nfs {

// One DFT pass along one axis of a complex array viewed as [outer][n][inner]
// (inner = 1: the axis is the contiguous one):
//   out[o][j][i] = scale * g[o][j][i] * sum_k in[o][k][i] exp(sign 2 pi i j k / n)
// with g = f (the filter, [L] in the array's own index order) or 1.
// A workgroup takes W columns (W consecutive inner indices of one o, or W
// consecutive lines when inner = 1) and J output rows j0 .. j0 + J - 1
// (blockIdx.y), stages the columns' n x W input block in LDS with loads that
// are contiguous across the columns (strided axes) or along each line
// (contiguous axis), and the n twiddle factors, computed in double
// precision.  Thread (j, c) forms one output with consecutive threads on
// consecutive columns, summing in float32 in order of k.
__global__ __launch_bounds__(256) void dft_axis_kernel(const float2* __restrict__ in, float2* __restrict__ out,
                                                       int64_t outer, int n, int64_t inner, int W, int J, int sign,
                                                       float scale, const float* __restrict__ f) {
  extern __shared__ float2 lds[];
  float2* tw = lds;                  // [n]
  float2* blk = lds + n;             // [n][W] inputs
  float2* ob = blk + (size_t)n * W;  // contiguous axis only: [J][W + 1] results
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)k / (double)n, &s, &c);
    tw[k] = make_float2((float)c, (float)(sign * s));
  }
  // columns of this workgroup: W lines from c0 (contiguous axis) or W inner
  // indices from c0 of line group o (strided axes)
  int64_t o = 0, c0, ncol;
  if (inner == 1) {
    c0 = (int64_t)blockIdx.x * W;
    ncol = outer - c0 < W ? outer - c0 : W;
  } else {
    const int64_t per = (inner + W - 1) / W;
    o = (int64_t)blockIdx.x / per;
    c0 = ((int64_t)blockIdx.x % per) * W;
    ncol = inner - c0 < W ? inner - c0 : W;
  }
  const int j0 = blockIdx.y * J;
  const int nj = n - j0 < J ? n - j0 : J;
  auto addr = [&](int k, int c) -> int64_t {
    return inner == 1 ? (c0 + c) * (int64_t)n + k : (o * (int64_t)n + k) * inner + c0 + c;
  };
  // loads: consecutive threads along each line (contiguous axis) or across
  // the columns (strided axes), i.e. contiguous in memory either way
  const int total = n * W;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int k, c;
    if (inner == 1) {
      c = e / n;
      k = e - c * n;
    } else {
      k = e / W;
      c = e - k * W;
    }
    blk[k * W + c] = c < ncol ? in[addr(k, c)] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int nout = J * W;
  for (int e = threadIdx.x; e < nout; e += blockDim.x) {
    const int jj = e / W, c = e - jj * W;
    if (c >= ncol || jj >= nj) continue;
    const int j = j0 + jj;
    float re = 0.f, im = 0.f;
    int idx = 0;  // (j k) mod n
    for (int k = 0; k < n; ++k) {
      const float2 x = blk[k * W + c], w = tw[idx];
      re = fmaf(x.x, w.x, re);
      re = fmaf(-x.y, w.y, re);
      im = fmaf(x.x, w.y, im);
      im = fmaf(x.y, w.x, im);
      idx += j;
      if (idx >= n) idx -= n;
    }
    if (inner == 1) {
      ob[jj * (W + 1) + c] = make_float2(re, im);
    } else {
      const int64_t a = addr(j, c);
      const float g = f ? f[a] * scale : scale;
      out[a] = make_float2(re * g, im * g);
    }
  }
  if (inner != 1) return;
  // contiguous axis: results leave along each line, as they came in
  __syncthreads();
  for (int e = threadIdx.x; e < nout; e += blockDim.x) {
    const int c = e / J, jj = e - c * J;
    if (c >= ncol || jj >= nj) continue;
    const int64_t a = addr(j0 + jj, c);
    const float g = f ? f[a] * scale : scale;
    const float2 v = ob[jj * (W + 1) + c];
    out[a] = make_float2(v.x * g, v.y * g);
  }
}

// out = rho * f * scale elementwise (the filter of a single-bin grid)
__global__ void filter_scale_kernel(const float2* __restrict__ in, float2* __restrict__ out, const float* f,
                                    float scale, int64_t L) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  const float g = f[l] * scale;
  out[l] = make_float2(in[l].x * g, in[l].y * g);
}

// Tiling of a pass: J output rows (32, or n if shorter) times W columns per
// workgroup, W * J <= 256 (one output per thread), W limited so that the
// twiddles, the n x W input block and, for the contiguous axis, the
// J x (W + 1) results fit in 64 KiB of LDS (n <= kMaxDftAxis = 2048).
static void dft_axis_tiling(int n, bool contiguous, int* W, int* J) {
  const int j = n < 32 ? n : 32;
  int w = 256 / j;
  const int slots = 65536 / 8 - n;  // float2 slots left after the twiddles
  while (w > 1 && n * w + (contiguous ? j * (w + 1) : 0) > slots) --w;
  *W = w;
  *J = j;
}

hipError_t launch_dft_axis(const float2* in, float2* out, int64_t outer, int n, int64_t inner, int sign, float scale,
                           const float* f, hipStream_t s) {
  const bool contiguous = inner == 1;
  int W, J;
  dft_axis_tiling(n, contiguous, &W, &J);
  const int64_t blocks = contiguous ? cdiv(outer, W) : outer * cdiv(inner, W);
  if (blocks == 0) return hipSuccess;
  const size_t lds = ((size_t)n + (size_t)n * W + (contiguous ? (size_t)J * (W + 1) : 0)) * sizeof(float2);
  hipLaunchKernelGGL(dft_axis_kernel, dim3((unsigned)blocks, (unsigned)cdiv(n, J)), dim3(256), lds, s, in, out, outer,
                     n, inner, W, J, sign, scale, f);
  return hipGetLastError();
}

hipError_t launch_filter_scale(const float2* in, float2* out, const float* f, float scale, int64_t L, hipStream_t s) {
  if (L == 0) return hipSuccess;
  hipLaunchKernelGGL(filter_scale_kernel, dim3((unsigned)cdiv(L, 256)), dim3(256), 0, s, in, out, f, scale, L);
  return hipGetLastError();
}

}  // namespace nfs
