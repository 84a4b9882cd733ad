// Conjugate-gradient vector kernels with float64 scalars kept on the device.
//
// CG on the normal equations E^H E rho = E^H sigma as in the paper's
// reconstruction-algorithm figure: r_0 = p_0 = E^H sigma, rho_0 = 0, and per
// iteration q = E^H E p, beta = p^H q, rho += (alpha/beta) p,
// r -= (alpha/beta) q, alpha' = r^H r, p = r + (alpha'/alpha) p.
//
// Determinism: every dot product is accumulated in float64 per thread, then
// per workgroup in a fixed tree, and the per-workgroup partials (at most
// kCgBlocks) are summed by every consumer workgroup in the same fixed tree,
// so every workgroup sees bit-identical scalars and runs are reproducible.
// No host synchronisation: a device stop flag, set when the loop ends
// (breakdown, exact convergence, tolerance), makes every later kernel of the
// solve return at once.
#include "nfs_internal.h"

namespace nfs {

enum { CG_MAXITER = 1, CG_TOL = 2, CG_EXACT = 3, CG_BREAKDOWN = 4 };

// A workgroup's place in the grid of one solve's vector kernel: column x,
// row y, and the grid's width nx (the solve's nblk).  A single-solve launch
// takes its own blockIdx and gridDim; a batched launch takes the slice from
// blockIdx.z and runs, for each slice, exactly the workgroups of that
// slice's own single-solve grid, so every slice's arithmetic and every
// fixed-order sum is that of its single solve.
struct Blk {
  int x, y, nx;
};
__device__ __forceinline__ Blk own_blk() { return Blk{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x}; }

// Sum of v over the workgroup (256 threads), fixed order; result in all threads.
__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Sum of the nblk partials part[0..nblk) in a fixed tree; result in all threads.
__device__ double sum_partials(const double* part, int nblk, double* red) {
  return block_sum((int)threadIdx.x < nblk ? part[threadIdx.x] : 0.0, red);
}

// Bound on the FP16 E operand entries S[c][l] p[l] of the new direction:
// workgroup maximum of smax[l] |p[l]| (smax[l] = max_c |S[c][l]|) into
// bmax[bx] (bx: the workgroup's column), the entries past the CG grid
// cleared by workgroup 0, so
// that the E operand packing (which reads all kBmaxBlocks entries) needs no
// pass of its own.  The bound is at most sqrt(2) above the largest |re| or
// |im|, which only moves the power-of-two scale.
__device__ void direction_bound(const CgState& st, float mx, float* redf, int bx) {
  redf[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) redf[threadIdx.x] = fmaxf(redf[threadIdx.x], redf[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) st.bmax[bx] = redf[0];
  if (bx == 0)
    for (int i = st.nblk + threadIdx.x; i < kBmaxBlocks; i += 256) st.bmax[i] = 0.f;
}

__device__ __forceinline__ float2 sum_splits(const float2* hpart, int nsplit, int64_t stride, int64_t l, float u) {
  const float2 v = sum_strided(hpart + l, nsplit, stride);
  return make_float2(v.x * u, v.y * u);
}

// smax[l] = max_c |S[c][l]|
__global__ void sens_absmax_kernel(const float2* __restrict__ sens, int G, int64_t L, float* __restrict__ smax) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  float m = 0.f;
  for (int c = 0; c < G; ++c) {
    const float2 v = sens[(int64_t)c * L + l];
    m = fmaxf(m, sqrtf(v.x * v.x + v.y * v.y));
  }
  smax[l] = m;
}

__global__ void cg_reset_kernel(int* stop, int* info) {
  *stop = 0;
  info[0] = 0;
  info[1] = 0;
}

__global__ __launch_bounds__(256) void cg_norm_m_kernel(const float2* __restrict__ m, int64_t n,
                                                        double* __restrict__ part) {
  __shared__ double red[256];
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float2 v = m[i];
    a += (double)v.x * v.x + (double)v.y * v.y;
  }
  a = block_sum(a, red);
  if (threadIdx.x == 0) part[blockIdx.x] = a;
}

// b = r = p = E^H m (sum of split partials), rho = 0, partial r^H r -> part[1]
__global__ __launch_bounds__(256) void cg_init_kernel(CgState st, const float2* __restrict__ hpart, int nsplit,
                                                      int64_t stride, const float* __restrict__ unscale,
                                                      float2* __restrict__ rho, int64_t L) {
  __shared__ double red[256];
  __shared__ float redf[256];
  const float u = unscale ? *unscale : 1.f;
  double a = 0.0;
  float mx = 0.f;
  for (int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x; l < L; l += (int64_t)gridDim.x * 256) {
    const float2 v = sum_splits(hpart, nsplit, stride, l, u);
    st.b[l] = v;
    st.r[l] = v;
    st.p[l] = v;
    rho[l] = make_float2(0.f, 0.f);
    if (st.iters) st.iters[l] = make_float2(0.f, 0.f);
    a += (double)v.x * v.x + (double)v.y * v.y;
    if (st.smax) mx = fmaxf(mx, st.smax[l] * sqrtf(v.x * v.x + v.y * v.y));
  }
  a = block_sum(a, red);
  if (threadIdx.x == 0) st.part[kCgBlocks + blockIdx.x] = a;
  if (st.smax) direction_bound(st, mx, redf, blockIdx.x);
}

// alpha_0, ||m||^2, hist row 0, early exit when E^H m == 0
__global__ __launch_bounds__(256) void cg_start_kernel(CgState st, int nblk_m, int n_iter) {
  __shared__ double red[256];
  const double a0 = sum_partials(st.part + kCgBlocks, st.nblk, red);
  const double d2 = sum_partials(st.part + 3 * kCgBlocks, nblk_m, red);
  if (threadIdx.x == 0) {
    st.alpha[0] = a0;
    st.scal[1] = d2;
    st.hist[0] = sqrt(a0);
    st.hist[1] = 0.0;
    st.hist[2] = d2;
    st.info[0] = 0;
    if (!(a0 > 0.0)) {  // zero or non-finite
      st.info[1] = (a0 == 0.0) ? CG_EXACT : CG_BREAKDOWN;
      *st.stop = 1;
    } else if (n_iter == 0) {
      st.info[1] = CG_MAXITER;
      *st.stop = 1;
    }
  }
}

// q = E^H E p (sum of split partials), partial Re p^H q -> part[0]
__device__ __forceinline__ void cg_beta_body(const CgState& st, const float2* __restrict__ hpart, int nsplit,
                                             int64_t stride, const float* __restrict__ unscale, int64_t L, Blk b) {
  if (*st.stop) return;
  __shared__ double red[256];
  const float u = unscale ? *unscale : 1.f;
  double a = 0.0;
  for (int64_t l = (int64_t)b.x * 256 + threadIdx.x; l < L; l += (int64_t)b.nx * 256) {
    const float2 q = sum_splits(hpart, nsplit, stride, l, u);
    const float2 p = st.p[l];
    st.q[l] = q;
    a += (double)p.x * q.x + (double)p.y * q.y;
  }
  a = block_sum(a, red);
  if (threadIdx.x == 0) st.part[b.x] = a;
}

__global__ __launch_bounds__(256) void cg_beta_kernel(CgState st, const float2* __restrict__ hpart, int nsplit,
                                                      int64_t stride, const float* __restrict__ unscale,
                                                      int64_t L) {
  cg_beta_body(st, hpart, nsplit, stride, unscale, L, own_blk());
}

// Partial sums, over the elements of workgroup column b.x, of
// conj(v_j) r for the stored residuals v_j, j in [j0, j1) (re-orthogonal-
// isation), into rpart.  r[l] is given by rfun(l).  Wave w takes j = j0 + w,
// j0 + w + 4, ...: each lane accumulates in float64 over its elements (in
// element order) and the wave reduces with a fixed xor-shuffle tree.
template <class RF>
__device__ void reorth_dots(const CgState& st, int j0, int j1, Blk b, RF&& rfun) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = j0 + wave; j < j1; j += kWaves) {
    const float2* v = st.V + (size_t)j * st.L;
    double re = 0.0, im = 0.0;
    for (int64_t base = (int64_t)b.x * 256; base < st.L; base += (int64_t)b.nx * 256)
      for (int k = lane; k < 256; k += 64) {
        const int64_t l = base + k;
        if (l >= st.L) break;
        const float2 a = v[l], r = rfun(l);
        re += (double)a.x * r.x + (double)a.y * r.y;
        im += (double)a.x * r.y - (double)a.y * r.x;
      }
    for (int off = 32; off > 0; off >>= 1) {
      re += __shfl_xor(re, off);
      im += __shfl_xor(im, off);
    }
    if (lane == 0) {
      st.rpart[(2 * (size_t)j) * kCgBlocks + b.x] = re;
      st.rpart[(2 * (size_t)j + 1) * kCgBlocks + b.x] = im;
    }
  }
}

// rho += gamma p, r -= gamma q with gamma = alpha_n / beta.  Grid
// (nblk, ny).  Row y = 0 does the update: rho, and the new r into st.r
// (partial r^H r -> part[1]) or, with re-orthogonalisation (nv > 0), into
// st.rn, left for cg_reorth_apply; partial ||rho||^2 -> part[2].  With
// nv > 0 every workgroup (x, y) also forms the partial dot products of the
// new r with v_j, j in [4y, 4y + 4), recomputing the new r of its elements
// from the unmodified r and q with the same arithmetic.
__device__ __forceinline__ void cg_update_body(const CgState& st, float2* __restrict__ rho, int64_t L, int n, int nv,
                                               Blk b) {
  if (*st.stop) return;
  __shared__ double red[256];
  const double beta = sum_partials(st.part, st.nblk, red);
  const double alpha = st.alpha[n];
  if (!(beta > 0.0) || !isfinite(beta)) {
    if (b.x == 0 && b.y == 0 && threadIdx.x == 0) {
      st.info[1] = CG_BREAKDOWN;
      *st.stop = 1;
    }
    return;
  }
  const double gamma = alpha / beta;
  const float gf = (float)gamma;
  if (b.y == 0) {
    float2* rout = nv > 0 ? st.rn : st.r;
    double a = 0.0, xx = 0.0;
    for (int64_t l = (int64_t)b.x * 256 + threadIdx.x; l < L; l += (int64_t)b.nx * 256) {
      const float2 p = st.p[l], q = st.q[l];
      float2 x = rho[l], r = st.r[l];
      x.x = fmaf(gf, p.x, x.x);
      x.y = fmaf(gf, p.y, x.y);
      r.x = fmaf(-gf, q.x, r.x);
      r.y = fmaf(-gf, q.y, r.y);
      rho[l] = x;
      rout[l] = r;
      if (st.iters) {
        const float j = st.icorr ? st.icorr[l] : 1.f;
        st.iters[(size_t)(n + 1) * L + l] = make_float2(x.x * j, x.y * j);
      }
      a += (double)r.x * r.x + (double)r.y * r.y;
      xx += (double)x.x * x.x + (double)x.y * x.y;
    }
    a = block_sum(a, red);
    xx = block_sum(xx, red);
    if (threadIdx.x == 0) {
      st.part[kCgBlocks + b.x] = a;
      st.part[2 * kCgBlocks + b.x] = xx;
      if (b.x == 0) st.scal[0] = beta;
    }
  }
  if (nv > 0) {
    const int j0 = 4 * b.y, j1 = j0 + 4 < nv ? j0 + 4 : nv;
    reorth_dots(st, j0, j1, b, [&](int64_t l) {
      const float2 q = st.q[l];
      float2 r = st.r[l];
      r.x = fmaf(-gf, q.x, r.x);
      r.y = fmaf(-gf, q.y, r.y);
      return r;
    });
  }
}

__global__ __launch_bounds__(256) void cg_update_kernel(CgState st, float2* __restrict__ rho, int64_t L, int n,
                                                        int nv) {
  cg_update_body(st, rho, L, n, nv, own_blk());
}

// residual replacement: r = b - (E^H E rho); partial r^H r -> part[1]
// (with nv > 0 also the re-orthogonalisation dot products of the new r)
__global__ __launch_bounds__(256) void cg_replace_kernel(CgState st, const float2* __restrict__ hpart, int nsplit,
                                                         int64_t stride, const float* __restrict__ unscale,
                                                         int64_t L, int nv) {
  if (*st.stop) return;
  __shared__ double red[256];
  const float u = unscale ? *unscale : 1.f;
  double a = 0.0;
  for (int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x; l < L; l += (int64_t)gridDim.x * 256) {
    const float2 ax = sum_splits(hpart, nsplit, stride, l, u);
    const float2 b = st.b[l];
    const float2 r = make_float2(b.x - ax.x, b.y - ax.y);
    st.r[l] = r;
    a += (double)r.x * r.x + (double)r.y * r.y;
  }
  a = block_sum(a, red);
  if (threadIdx.x == 0) st.part[kCgBlocks + blockIdx.x] = a;
  if (nv > 0) {
    __syncthreads();  // this workgroup's r writes are visible to all its waves
    reorth_dots(st, 0, nv, own_blk(), [&](int64_t l) { return st.r[l]; });
  }
}

// alpha_{n+1} = r^H r; p = r + (alpha_{n+1} / alpha_n) p; with
// re-orthogonalisation also V[n+1] = r / sqrt(alpha_{n+1}).  Workgroup 0
// writes history row n+1 (||rho_{n+1}|| from the partials of cg_update) and
// takes the stop decision.  It raises the stop flag itself: a workgroup of
// this launch that starts after that skips its share of the p and V
// updates, which is harmless because neither is read once the loop stops.
__device__ __forceinline__ void cg_direction_body(const CgState& st, int64_t L, int n, int n_iter, double tol, Blk b) {
  if (*st.stop) return;
  __shared__ double red[256];
  const double anew = sum_partials(st.part + kCgBlocks, st.nblk, red);
  const double aold = st.alpha[n];
  const float bf = (float)(anew / aold);
  const bool store = st.V && anew > 0.0 && isfinite(anew);
  const float inv = store ? (float)(1.0 / sqrt(anew)) : 0.f;
  float2* v = store ? st.V + (size_t)(n + 1) * L : nullptr;
  float mx = 0.f;
  for (int64_t l = (int64_t)b.x * 256 + threadIdx.x; l < L; l += (int64_t)b.nx * 256) {
    const float2 r = st.r[l];
    float2 p = st.p[l];
    p.x = fmaf(bf, p.x, r.x);
    p.y = fmaf(bf, p.y, r.y);
    st.p[l] = p;
    if (store) v[l] = make_float2(r.x * inv, r.y * inv);
    if (st.smax) mx = fmaxf(mx, st.smax[l] * sqrtf(p.x * p.x + p.y * p.y));
  }
  if (st.smax) {
    __shared__ float redf[256];
    direction_bound(st, mx, redf, b.x);
  }
  if (b.x != 0) return;
  const double xx = sum_partials(st.part + 2 * kCgBlocks, st.nblk, red);
  if (threadIdx.x != 0) return;
  const double beta = st.scal[0];
  const double d2 = st.scal[1] - aold * aold / beta;
  st.scal[1] = d2;
  st.alpha[n + 1] = anew;
  double* h = st.hist + 3 * (size_t)(n + 1);
  h[0] = sqrt(anew);
  h[1] = sqrt(xx);
  h[2] = d2;
  st.info[0] = n + 1;
  int status = 0;
  if (!isfinite(anew)) status = CG_BREAKDOWN;
  else if (anew == 0.0) status = CG_EXACT;
  else if (tol > 0.0 && sqrt(anew) <= tol * sqrt(st.alpha[0])) status = CG_TOL;
  else if (n + 1 >= n_iter) status = CG_MAXITER;
  if (status) {
    st.info[1] = status;
    *st.stop = 1;
  }
}

__global__ __launch_bounds__(256) void cg_direction_kernel(CgState st, int64_t L, int n, int n_iter, double tol) {
  cg_direction_body(st, L, n, n_iter, tol, own_blk());
}

// ---------------------------------------------------------------------------
// Re-orthogonalisation of the residual against the stored normalised
// residuals v_j (classical Gram-Schmidt with float64 dot products).
__global__ __launch_bounds__(256) void cg_store_v_kernel(CgState st, int j) {
  if (*st.stop) return;
  const double a = st.alpha[j];
  if (!(a > 0.0)) return;
  const float inv = (float)(1.0 / sqrt(a));
  float2* v = st.V + (size_t)j * st.L;
  for (int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x; l < st.L; l += (int64_t)gridDim.x * 256) {
    const float2 r = st.r[l];
    v[l] = make_float2(r.x * inv, r.y * inv);
  }
}

// r = src - sum_j (v_j^H src) v_j with src = st.rn (after cg_update) or st.r
// (after a residual replacement).  Every workgroup first sums the nblk
// partials of each v_j^H src itself (thread i takes sum i, partials in
// workgroup order), so all workgroups use bit-identical coefficients;
// partial r^H r -> part[1].
__device__ __forceinline__ void cg_reorth_apply_body(const CgState& st, int nv, int from_rn, Blk b) {
  if (*st.stop) return;
  __shared__ double red[256];
  __shared__ double coef[2 * (kMaxReorth + 1)];
  // (both loops issue the loads of several terms before using them in
  // order, so the arithmetic is that of the plain loops)
  for (int i = threadIdx.x; i < 2 * nv; i += 256) {
    const double* pp = st.rpart + (size_t)i * kCgBlocks;
    double t = 0.0;
    for (int b0 = 0; b0 < st.nblk; b0 += 8) {
      double w[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) w[k] = b0 + k < st.nblk ? pp[b0 + k] : 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (b0 + k < st.nblk) t += w[k];
    }
    coef[i] = t;
  }
  __syncthreads();
  double a = 0.0;
  for (int64_t l = (int64_t)b.x * 256 + threadIdx.x; l < st.L; l += (int64_t)b.nx * 256) {
    float2 r = from_rn ? st.rn[l] : st.r[l];
    for (int j0 = 0; j0 < nv; j0 += 4) {
      float2 v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = j0 + k < nv ? st.V[(size_t)(j0 + k) * st.L + l] : make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (j0 + k < nv) {
          const float cr = (float)coef[2 * (j0 + k)], ci = (float)coef[2 * (j0 + k) + 1];
          r.x -= cr * v[k].x - ci * v[k].y;
          r.y -= cr * v[k].y + ci * v[k].x;
        }
    }
    st.r[l] = r;
    a += (double)r.x * r.x + (double)r.y * r.y;
  }
  a = block_sum(a, red);
  if (threadIdx.x == 0) st.part[kCgBlocks + b.x] = a;
}

__global__ __launch_bounds__(256) void cg_reorth_apply_kernel(CgState st, int nv, int from_rn) {
  cg_reorth_apply_body(st, nv, from_rn, own_blk());
}

// ---------------------------------------------------------------------------
// Batched forms for the lock-step batched solve: one launch runs a step for
// every slice.  Grid (max nblk, rows, slices); the slice's arguments are
// read from the device array sl (written once per solve), and the
// workgroups past the slice's own nblk return at once.
__device__ __forceinline__ bool slice_blk(const CgSlice* __restrict__ sl, CgSlice& a, Blk& b) {
  a = sl[blockIdx.z];
  b = Blk{(int)blockIdx.x, (int)blockIdx.y, a.st.nblk};
  return b.x < b.nx;
}

__global__ __launch_bounds__(256) void cg_beta_batched_kernel(const CgSlice* __restrict__ sl) {
  CgSlice a;
  Blk b;
  if (slice_blk(sl, a, b)) cg_beta_body(a.st, a.hpart, a.nsplit, a.stride, a.unscale, a.st.L, b);
}

__global__ __launch_bounds__(256) void cg_update_batched_kernel(const CgSlice* __restrict__ sl, int n, int nv) {
  CgSlice a;
  Blk b;
  if (slice_blk(sl, a, b)) cg_update_body(a.st, a.rho, a.st.L, n, nv, b);
}

__global__ __launch_bounds__(256) void cg_reorth_apply_batched_kernel(const CgSlice* __restrict__ sl, int nv,
                                                                      int from_rn) {
  CgSlice a;
  Blk b;
  if (slice_blk(sl, a, b)) cg_reorth_apply_body(a.st, nv, from_rn, b);
}

__global__ __launch_bounds__(256) void cg_direction_batched_kernel(const CgSlice* __restrict__ sl, int n, int n_iter,
                                                                   double tol) {
  CgSlice a;
  Blk b;
  if (slice_blk(sl, a, b)) cg_direction_body(a.st, a.st.L, n, n_iter, tol, b);
}

__global__ void store_slice_args_kernel(CgSlice cg, PackSlice pe, PackSlice ph, CgSlice* cg_out, PackSlice* pe_out,
                                        PackSlice* ph_out) {
  *cg_out = cg;
  *pe_out = pe;
  *ph_out = ph;
}

__global__ void cg_finish_kernel(float2* __restrict__ rho, const float* __restrict__ icorr, int64_t L) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  const float j = icorr[l];
  float2 x = rho[l];
  x.x *= j;
  x.y *= j;
  rho[l] = x;
}

// ---------------------------------------------------------------------------
hipError_t launch_cg_reset(const CgState& st, hipStream_t s) {
  hipLaunchKernelGGL(cg_reset_kernel, dim3(1), dim3(1), 0, s, st.stop, st.info);
  return hipGetLastError();
}

hipError_t launch_cg_norm_m(const CgState& st, const float2* m, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(cg_norm_m_kernel, dim3(kCgBlocks), dim3(256), 0, s, m, n, st.part + 3 * kCgBlocks);
  return hipGetLastError();
}

hipError_t launch_cg_init(const CgState& st, const float2* hpart, int nsplit, int64_t stride, const float* unscale,
                          float2* rho, int64_t L, hipStream_t s) {
  hipLaunchKernelGGL(cg_init_kernel, dim3(st.nblk), dim3(256), 0, s, st, hpart, nsplit, stride, unscale, rho, L);
  return hipGetLastError();
}

hipError_t launch_sens_absmax(const float2* sens, int G, int64_t L, float* smax, hipStream_t s) {
  if (L == 0) return hipSuccess;
  hipLaunchKernelGGL(sens_absmax_kernel, dim3((unsigned)cdiv(L, 256)), dim3(256), 0, s, sens, G, L, smax);
  return hipGetLastError();
}

hipError_t launch_cg_start(const CgState& st, int n_iter, hipStream_t s) {
  hipLaunchKernelGGL(cg_start_kernel, dim3(1), dim3(256), 0, s, st, kCgBlocks, n_iter);
  return hipGetLastError();
}

hipError_t launch_cg_beta(const CgState& st, const float2* hpart, int nsplit, int64_t stride, const float* unscale,
                          int64_t L, hipStream_t s) {
  hipLaunchKernelGGL(cg_beta_kernel, dim3(st.nblk), dim3(256), 0, s, st, hpart, nsplit, stride, unscale, L);
  return hipGetLastError();
}

hipError_t launch_cg_update(const CgState& st, float2* rho, int64_t L, int n, int nv, hipStream_t s) {
  const unsigned ny = nv > 0 ? (unsigned)cdiv(nv, 4) : 1u;
  hipLaunchKernelGGL(cg_update_kernel, dim3(st.nblk, ny), dim3(256), 0, s, st, rho, L, n, nv);
  return hipGetLastError();
}

hipError_t launch_cg_replace(const CgState& st, const float2* hpart, int nsplit, int64_t stride,
                             const float* unscale, int64_t L, int nv, hipStream_t s) {
  hipLaunchKernelGGL(cg_replace_kernel, dim3(st.nblk), dim3(256), 0, s, st, hpart, nsplit, stride, unscale, L, nv);
  return hipGetLastError();
}

hipError_t launch_cg_direction(const CgState& st, int64_t L, int n, int n_iter, double tol, hipStream_t s) {
  hipLaunchKernelGGL(cg_direction_kernel, dim3(st.nblk), dim3(256), 0, s, st, L, n, n_iter, tol);
  return hipGetLastError();
}

hipError_t launch_cg_store_v(const CgState& st, int j, hipStream_t s) {
  hipLaunchKernelGGL(cg_store_v_kernel, dim3(st.nblk), dim3(256), 0, s, st, j);
  return hipGetLastError();
}

hipError_t launch_cg_reorth_apply(const CgState& st, int nv, bool from_rn, hipStream_t s) {
  hipLaunchKernelGGL(cg_reorth_apply_kernel, dim3(st.nblk), dim3(256), 0, s, st, nv, (int)from_rn);
  return hipGetLastError();
}

hipError_t launch_store_slice_args(const CgSlice& cg, const PackSlice& pe, const PackSlice& ph, CgSlice* cg_out,
                                   PackSlice* pe_out, PackSlice* ph_out, hipStream_t s) {
  hipLaunchKernelGGL(store_slice_args_kernel, dim3(1), dim3(1), 0, s, cg, pe, ph, cg_out, pe_out, ph_out);
  return hipGetLastError();
}

hipError_t launch_cg_beta_batched(const CgSlice* sl, int n, int max_nblk, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cg_beta_batched_kernel, dim3(max_nblk, 1, n), dim3(256), 0, s, sl);
  return hipGetLastError();
}

hipError_t launch_cg_update_batched(const CgSlice* sl, int n, int max_nblk, int it, int nv, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned ny = nv > 0 ? (unsigned)cdiv(nv, 4) : 1u;
  hipLaunchKernelGGL(cg_update_batched_kernel, dim3(max_nblk, ny, n), dim3(256), 0, s, sl, it, nv);
  return hipGetLastError();
}

hipError_t launch_cg_reorth_apply_batched(const CgSlice* sl, int n, int max_nblk, int nv, bool from_rn,
                                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cg_reorth_apply_batched_kernel, dim3(max_nblk, 1, n), dim3(256), 0, s, sl, nv, (int)from_rn);
  return hipGetLastError();
}

hipError_t launch_cg_direction_batched(const CgSlice* sl, int n, int max_nblk, int it, int n_iter, double tol,
                                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cg_direction_batched_kernel, dim3(max_nblk, 1, n), dim3(256), 0, s, sl, it, n_iter, tol);
  return hipGetLastError();
}

hipError_t launch_cg_finish(const CgState& st, float2* rho, const float* icorr, int64_t L, hipStream_t s) {
  (void)st;
  if (!icorr || L == 0) return hipSuccess;
  hipLaunchKernelGGL(cg_finish_kernel, dim3((unsigned)cdiv(L, 256)), dim3(256), 0, s, rho, icorr, L);
  return hipGetLastError();
}

// out[c][k] = m[c][k] * exp(i sign theta[k]): the per-sample phase offset
// that a compressed phase basis moves out of the tile phase.  One thread
// per sample; the rotation is evaluated in double precision once per sample
// and applied to every coil (in place when out == m).
__global__ __launch_bounds__(256) void phase_shift_kernel(const float2* m, float2* out, const double* __restrict__ theta,
                                                          int G, int64_t K, int sign) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= K) return;
  double sn, cs;
  sincos((double)sign * theta[k], &sn, &cs);
  for (int c = 0; c < G; ++c) {
    const float2 v = m[(int64_t)c * K + k];
    out[(int64_t)c * K + k] = make_float2((float)(cs * v.x - sn * v.y), (float)(sn * v.x + cs * v.y));
  }
}

hipError_t launch_phase_shift(const float2* m, float2* out, const double* theta, int G, int64_t K, int sign,
                              hipStream_t s) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(phase_shift_kernel, dim3((unsigned)cdiv(K, 256)), dim3(256), 0, s, m, out, theta, G, K, sign);
  return hipGetLastError();
}

}  // namespace nfs
