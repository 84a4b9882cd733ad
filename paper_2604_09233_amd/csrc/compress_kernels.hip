// Phase-basis compression on the device: the computation of the host call
// nfs_compress_basis (see capi.hip), in double precision, for bases that
// live in device memory, so that a new geometry (kcoef is measured per scan)
// costs a few short launches instead of host copies and host arithmetic.
//
// phi(k, l) = sum_b a_b(k) h_b(l) over T = P + 1 terms (a_0 = t, h_0 = b0).
// With s_b = max_k |a_b|, the scaled rows h^_b = s_b h_b, their means mu_b
// and the centred rows A_b = h^_b - mu_b:
//   phi = theta(k) + sum_b (a_b / s_b)(k) A_b(l),  theta = sum_b (a_b / s_b) mu_b;
// the eigenvectors U of the Gram matrix A A^T (largest eigenvalue first) give
// directions h'_j = sum_b U_bj A_b (voxel side) and a'_j = sum_b (a_b / s_b)
// U_bj (sample side); the first r* directions are kept, r* the smallest
// count whose residual E_b = A_b - sum_{j < r*} U_bj h'_j satisfies
//   max_l sum_b |E_b(l)| <= rel_tol * sum_b max|a_b| max|h_b|.
// Sums over voxels are formed per workgroup and added in workgroup order
// (fixed order: results are reproducible run to run).
#include "nfs_internal.h"

namespace nfs {

namespace {

// coefficients of term b: a_b(k) (sample side) and h_b(l) (voxel side)
__device__ __forceinline__ double a_coef(const float* t, const float* kcoef, int P, int b, int64_t k) {
  return b == 0 ? (double)t[k] : (double)kcoef[k * P + (b - 1)];
}
__device__ __forceinline__ double h_coef(const float* b0, const float* fields, int64_t L, int b, int64_t l) {
  return b == 0 ? (double)b0[l] : (double)fields[(int64_t)(b - 1) * L + l];
}
// s_b = max_k |a_b(k)| from the term maxima (float bits, exact)
__device__ __forceinline__ double s_of(const unsigned* tmax, int b) { return (double)__uint_as_float(tmax[b]); }

// Workgroup sum of one double per thread, thread 0 gets the result (fixed
// order: lane pairs by shuffle, then the four waves in order).
__device__ double block_sum_d(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

}  // namespace

// Per-workgroup partial sums of the scaled rows: part[blk][b] = sum over
// the workgroup's voxels of s_b h_b(l).
__global__ __launch_bounds__(256) void cmp_mean_kernel(const float* __restrict__ b0, const float* __restrict__ fields,
                                                       int64_t L, int T, const unsigned* __restrict__ tmax,
                                                       double* __restrict__ part) {
  __shared__ double red[4];
  for (int b = 0; b < T; ++b) {
    const double s = s_of(tmax, b);
    double acc = 0.0;
    for (int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x; l < L; l += (int64_t)gridDim.x * 256)
      acc += s * h_coef(b0, fields, L, b, l);
    const double tot = block_sum_d(acc, red);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * T + b] = tot;
  }
}

// Per-workgroup partial Gram matrix of the centred rows (upper triangle,
// pair index p * T + q for p <= q): part[blk][p * T + q].  mu from the sums
// of the previous pass, added in workgroup order by every thread.
__global__ __launch_bounds__(256) void cmp_gram_kernel(const float* __restrict__ b0, const float* __restrict__ fields,
                                                       int64_t L, int T, const unsigned* __restrict__ tmax,
                                                       const double* __restrict__ mean_part, int nblk,
                                                       double* __restrict__ part) {
  __shared__ double red[4];
  __shared__ double mu[kMaxTerms], sc[kMaxTerms];
  if ((int)threadIdx.x < T) {
    double m = 0.0;
    for (int i = 0; i < nblk; ++i) m += mean_part[(int64_t)i * T + threadIdx.x];
    mu[threadIdx.x] = L > 0 ? m / (double)L : 0.0;
    sc[threadIdx.x] = s_of(tmax, threadIdx.x);
  }
  __syncthreads();
  for (int p = 0; p < T; ++p)
    for (int q = p; q < T; ++q) {
      double acc = 0.0;
      for (int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x; l < L; l += (int64_t)gridDim.x * 256) {
        const double ap = sc[p] * h_coef(b0, fields, L, p, l) - mu[p];
        const double aq = sc[q] * h_coef(b0, fields, L, q, l) - mu[q];
        acc += ap * aq;
      }
      const double tot = block_sum_d(acc, red);
      if (threadIdx.x == 0) part[(int64_t)blockIdx.x * T * T + p * T + q] = tot;
    }
}

// One wave: the Gram matrix (partials added in workgroup order), its
// eigenvectors by cyclic Jacobi rotations (the rotation that zeroes S[p][q],
// tan = the smaller root, as in the host computation; lane k updates row and
// column entries k), sorted by descending eigenvalue.  Writes
// U [T][T] (column j = direction j), mu [T], and s [T] into `eig`:
// eig[0 .. T*T) = U, eig[T*T .. T*T+T) = mu, eig[T*T+T .. T*T+2T) = s.
__global__ __launch_bounds__(64) void cmp_eigen_kernel(int64_t L, int T, const unsigned* __restrict__ tmax,
                                                       const double* __restrict__ mean_part,
                                                       const double* __restrict__ gram_part, int nblk,
                                                       double* __restrict__ eig) {
  __shared__ double S[kMaxTerms][kMaxTerms + 1];
  __shared__ double V[kMaxTerms][kMaxTerms + 1];
  __shared__ int order[kMaxTerms];
  const int k = threadIdx.x;
  if (k < T) {
    double m = 0.0;
    for (int i = 0; i < nblk; ++i) m += mean_part[(int64_t)i * T + k];
    eig[T * T + k] = L > 0 ? m / (double)L : 0.0;
    eig[T * T + T + k] = s_of(tmax, k);
    for (int q = 0; q < T; ++q) {
      const int p0 = k < q ? k : q, q0 = k < q ? q : k;
      double g = 0.0;
      for (int i = 0; i < nblk; ++i) g += gram_part[(int64_t)i * T * T + p0 * T + q0];
      S[k][q] = g;
      V[k][q] = k == q ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, diag = 0.0;
    if (k < T) {
      diag = S[k][k] * S[k][k];
      for (int q = k + 1; q < T; ++q) off += S[k][q] * S[k][q];
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      diag += __shfl_xor(diag, o);
    }
    if (off <= 1e-34 * diag || off == 0.0) break;
    for (int p = 0; p < T; ++p)
      for (int q = p + 1; q < T; ++q) {
        const double apq = S[p][q];
        if (apq == 0.0) continue;  // uniform across the wave
        const double app = S[p][p], aqq = S[q][q];
        const double zeta = (aqq - app) / (2.0 * apq);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        __syncthreads();
        if (k < T) {  // columns p, q
          const double skp = S[k][p], skq = S[k][q];
          S[k][p] = c * skp - s * skq;
          S[k][q] = s * skp + c * skq;
        }
        __syncthreads();
        if (k < T) {  // rows p, q
          const double spk = S[p][k], sqk = S[q][k];
          S[p][k] = c * spk - s * sqk;
          S[q][k] = s * spk + c * sqk;
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
        __syncthreads();
      }
  }
  if (k == 0) {  // stable sort by descending eigenvalue
    for (int i = 0; i < T; ++i) order[i] = i;
    for (int i = 1; i < T; ++i) {
      const int v = order[i];
      int j = i - 1;
      while (j >= 0 && S[order[j]][order[j]] < S[v][v]) {
        order[j + 1] = order[j];
        --j;
      }
      order[j + 1] = v;
    }
  }
  __syncthreads();
  if (k < T)
    for (int j = 0; j < T; ++j) eig[k * T + j] = V[k][order[j]];
}

// Per voxel the residual bound after r kept directions, r = 0..T:
// res_r(l) = sum_b |A_b(l) - sum_{j < r} U_bj h'_j(l)|; per workgroup the
// maximum over its voxels: part[blk][r].
__global__ __launch_bounds__(256) void cmp_resid_kernel(const float* __restrict__ b0, const float* __restrict__ fields,
                                                        int64_t L, int T, const double* __restrict__ eig,
                                                        double* __restrict__ part) {
  __shared__ double U[kMaxTerms * kMaxTerms], mu[kMaxTerms], sc[kMaxTerms];
  __shared__ double red[kMaxTerms + 1][4];
  for (int i = threadIdx.x; i < T * T; i += 256) U[i] = eig[i];
  if ((int)threadIdx.x < T) {
    mu[threadIdx.x] = eig[T * T + threadIdx.x];
    sc[threadIdx.x] = eig[T * T + T + threadIdx.x];
  }
  __syncthreads();
  double worst[kMaxTerms + 1];
#pragma unroll
  for (int r = 0; r <= kMaxTerms; ++r) worst[r] = 0.0;
  for (int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x; l < L; l += (int64_t)gridDim.x * 256) {
    double A[kMaxTerms], E[kMaxTerms];
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < kMaxTerms; ++b)
      if (b < T) {
        A[b] = sc[b] * h_coef(b0, fields, L, b, l) - mu[b];
        E[b] = A[b];
        acc += fabs(E[b]);
      }
    worst[0] = fmax(worst[0], acc);
#pragma unroll
    for (int j = 0; j < kMaxTerms; ++j)
      if (j < T) {
        double h = 0.0;
#pragma unroll
        for (int b = 0; b < kMaxTerms; ++b)
          if (b < T) h += U[b * T + j] * A[b];
        acc = 0.0;
#pragma unroll
        for (int b = 0; b < kMaxTerms; ++b)
          if (b < T) {
            E[b] -= U[b * T + j] * h;
            acc += fabs(E[b]);
          }
        worst[j + 1] = fmax(worst[j + 1], acc);
      }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r <= kMaxTerms; ++r)
    if (r <= T) {
      double v = worst[r];
      for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
      if (lane == 0) red[r][wave] = v;
    }
  __syncthreads();
  if ((int)threadIdx.x <= T) {
    double v = red[threadIdx.x][0];
    for (int w = 1; w < 4; ++w) v = fmax(v, red[threadIdx.x][w]);
    part[(int64_t)blockIdx.x * (T + 1) + threadIdx.x] = v;
  }
}

// r* and the outputs' scalars: sel[0] = r* (as int bits), n_basis = max(r* -
// 1, 0), err_bound = the residual bound at r*.
__global__ void cmp_select_kernel(int T, const unsigned* __restrict__ tmax, const double* __restrict__ part, int nblk,
                                  double rel_tol, int* __restrict__ sel, int* __restrict__ n_basis_out,
                                  double* __restrict__ err_bound) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double bound = 0.0;
  for (int b = 0; b < T; ++b) bound += (double)__uint_as_float(tmax[b]) * (double)__uint_as_float(tmax[kMaxTerms + b]);
  const double tol = rel_tol * bound;
  int r = 0;
  double err = 0.0;
  for (r = 0; r <= T; ++r) {
    err = 0.0;
    for (int i = 0; i < nblk; ++i) err = fmax(err, part[(int64_t)i * (T + 1) + r]);
    if (err <= tol || r == T) break;
  }
  sel[0] = r;
  *n_basis_out = r > 0 ? r - 1 : 0;
  if (err_bound) *err_bound = err;
}

// Voxel side of the kept directions: b0_out = h'_0 (0 if none is kept),
// fields_out[j - 1] = h'_j for 1 <= j < r*.
__global__ __launch_bounds__(256) void cmp_out_voxel_kernel(const float* __restrict__ b0,
                                                            const float* __restrict__ fields, int64_t L, int T,
                                                            const double* __restrict__ eig, const int* __restrict__ sel,
                                                            float* __restrict__ b0_out, float* __restrict__ fields_out) {
  const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (l >= L) return;
  const int r = sel[0];
  const double* U = eig;
  double A[kMaxTerms];
#pragma unroll
  for (int b = 0; b < kMaxTerms; ++b)
    if (b < T) A[b] = eig[T * T + T + b] * h_coef(b0, fields, L, b, l) - eig[T * T + b];
  if (r == 0) b0_out[l] = 0.f;
  for (int j = 0; j < r; ++j) {
    double h = 0.0;
#pragma unroll
    for (int b = 0; b < kMaxTerms; ++b)
      if (b < T) h += U[b * T + j] * A[b];
    if (j == 0)
      b0_out[l] = (float)h;
    else
      fields_out[(int64_t)(j - 1) * L + l] = (float)h;
  }
}

// Sample side: theta = sum_b (a_b / s_b) mu_b, t_out = a'_0 (0 if none is
// kept), kcoef_out[k][j - 1] = a'_j for 1 <= j < r* (row stride r* - 1).
__global__ __launch_bounds__(256) void cmp_out_sample_kernel(const float* __restrict__ t,
                                                             const float* __restrict__ kcoef, int64_t K, int P,
                                                             const double* __restrict__ eig,
                                                             const int* __restrict__ sel, float* __restrict__ t_out,
                                                             float* __restrict__ kcoef_out,
                                                             double* __restrict__ theta) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= K) return;
  const int T = P + 1, r = sel[0];
  const int Pn = r > 0 ? r - 1 : 0;
  const double* U = eig;
  double as[kMaxTerms];
  double th = 0.0;
#pragma unroll
  for (int b = 0; b < kMaxTerms; ++b)
    if (b < T) {
      const double s = eig[T * T + T + b];
      as[b] = s > 0.0 ? a_coef(t, kcoef, P, b, k) / s : 0.0;
      th += as[b] * eig[T * T + b];
    }
  theta[k] = th;
  if (r == 0) t_out[k] = 0.f;
  for (int j = 0; j < r; ++j) {
    double v = 0.0;
#pragma unroll
    for (int b = 0; b < kMaxTerms; ++b)
      if (b < T) v += as[b] * U[b * T + j];
    if (j == 0)
      t_out[k] = (float)v;
    else
      kcoef_out[k * Pn + (j - 1)] = (float)v;
  }
}

// workgroups of the voxel reductions
static int cmp_blocks(int64_t L) {
  const int64_t b = cdiv(L, 256);
  return (int)(b < 1 ? 1 : (b > kCmpBlocks ? kCmpBlocks : b));
}

size_t compress_workspace_doubles(int64_t L, int P) {
  const int T = P + 1, nb = cmp_blocks(L);
  return (size_t)nb * T + (size_t)nb * T * T + (size_t)nb * (T + 1) + (size_t)T * T + 2 * (size_t)T + 2;
}

hipError_t launch_compress_basis(const float* fields, const float* b0, const float* kcoef, const float* t, int64_t L,
                                 int64_t K, int P, double rel_tol, const unsigned* tmax, double* ws,
                                 float* fields_out, float* b0_out, float* kcoef_out, float* t_out, double* theta,
                                 int* n_basis_out, double* err_bound, hipStream_t s) {
  const int T = P + 1, nb = cmp_blocks(L);
  double* mean_part = ws;
  double* gram_part = mean_part + (size_t)nb * T;
  double* res_part = gram_part + (size_t)nb * T * T;
  double* eig = res_part + (size_t)nb * (T + 1);
  int* sel = reinterpret_cast<int*>(eig + (size_t)T * T + 2 * T);
  hipLaunchKernelGGL(cmp_mean_kernel, dim3(nb), dim3(256), 0, s, b0, fields, L, T, tmax, mean_part);
  hipLaunchKernelGGL(cmp_gram_kernel, dim3(nb), dim3(256), 0, s, b0, fields, L, T, tmax, mean_part, nb, gram_part);
  hipLaunchKernelGGL(cmp_eigen_kernel, dim3(1), dim3(64), 0, s, L, T, tmax, mean_part, gram_part, nb, eig);
  hipLaunchKernelGGL(cmp_resid_kernel, dim3(nb), dim3(256), 0, s, b0, fields, L, T, eig, res_part);
  hipLaunchKernelGGL(cmp_select_kernel, dim3(1), dim3(64), 0, s, T, tmax, res_part, nb, rel_tol, sel, n_basis_out,
                     err_bound);
  if (L > 0)
    hipLaunchKernelGGL(cmp_out_voxel_kernel, dim3((unsigned)cdiv(L, 256)), dim3(256), 0, s, b0, fields, L, T, eig, sel,
                       b0_out, fields_out);
  if (K > 0)
    hipLaunchKernelGGL(cmp_out_sample_kernel, dim3((unsigned)cdiv(K, 256)), dim3(256), 0, s, t, kcoef, K, P, eig, sel,
                       t_out, kcoef_out, theta);
  return hipGetLastError();
}

}  // namespace nfs
