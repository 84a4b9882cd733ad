// Sensitivity and B0 map estimation from multi-echo prescan data (Methods,
// "Computation of sensitivity maps" and "Computation of B0 maps"), float64
// throughout.
//
// Initial sensitivities.  Per voxel the coil x echo matrix X (G <= 16 rows)
// has as first left singular vector the dominant eigenvector of the
// Hermitian Gram matrix X X^H.  The Gram matrix is formed on the float64
// matrix cores (16x16x4 tiles, echoes as the contraction index) and its
// dominant eigenvector isolated by repeated squaring: B <- B^2 / ||B||_F
// converges to the rank-one projector u u^H at the rate (l2 / l1)^(2^k).
// Because B is Hermitian, the operand layouts of the 16x16x4 instruction line
// up with its result layout (register r of a lane holds row lane/16 + 4 r of
// column lane % 16, which is, conjugated, the A operand and, as is, the B
// operand of the r-th four-wide slice of the contraction), so every squaring
// stays in registers.  u is read off the column of the largest diagonal entry and
// rotated so that its coil sum is real and non-negative.
//
// Smoothing.  Both smoothing equations are least-squares problems whose
// normal equations A x = b have a stencil matrix:
//   sensitivities: A = diag(t) + a sum_d D2_d^T diag(w) D2_d, t = M_T^2,
//                  w = M_R^2, b = M_T o (|S^|, Re n, Im n), n = S^/|S^|;
//   B0:            A = I + a sum_d D1_d^T diag(w) D1_d, w = eps^2, b = B0^.
// D2 along an axis has a row centred at every voxel whose two neighbours
// along it exist; D1 a row at every voxel whose next neighbour exists, the
// row weight taken at that voxel.  A is applied matrix-free and the systems
// (3G sensitivity right-hand sides share one A) are solved by Jacobi-
// preconditioned CG with float64 vectors and scalars, per right-hand side,
// with fixed-order reductions.  The search direction p = D^-1 r + beta p is
// not stored between the two passes of an iteration: the apply pass forms
// it at each stencil point from r and the previous p (the same expression
// everywhere, so the stored value and the one used in A p agree bitwise).
//
// B0 fit.  Per voxel the echoes are combined with the sensitivities,
// c_n = sum_c conj(S_c) x_cn / sum_c |S_c|^2, the phase of c_n conj(c_0)
// is unwrapped along n (a jump of at least pi between neighbouring echoes is
// taken modulo 2 pi into (-pi, pi]), and phi_n = a n + b mod(n, 2) is fitted
// by least squares (2x2 normal equations); B0^ = a / dTE, eps = the root mean
// square fit residual.
#include "nfs.h"
#include "nfs_internal.h"

#include <algorithm>

namespace nfs {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kVoxPerBlock = 16;  // voxels staged per workgroup, 4 per wave
constexpr int kEchoChunk = 16;    // echoes staged per pass
constexpr int kStageStride = kVoxPerBlock + 1;
constexpr int kMaxSquarings = 24;
constexpr double kProjTol = 1e-13;  // trace(B) - 1 below this: one more squaring, then stop

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// acc += Y Y^H for the 16 x 4 complex block Y held one entry per lane (row
// lane % 16, column lane / 16); acc in the 16x16x4 result layout.
__device__ __forceinline__ void herm_rank4(double yr, double yi, dbl4& ar, dbl4& ai) {
  ar = __builtin_amdgcn_mfma_f64_16x16x4f64(yr, yr, ar, 0, 0, 0);
  ar = __builtin_amdgcn_mfma_f64_16x16x4f64(yi, yi, ar, 0, 0, 0);
  ai = __builtin_amdgcn_mfma_f64_16x16x4f64(yi, yr, ai, 0, 0, 0);
  ai = __builtin_amdgcn_mfma_f64_16x16x4f64(-yr, yi, ai, 0, 0, 0);
}

// Row of the 16x16x4 float64 result held in register r of a lane (its
// column is lane % 16).
__device__ __forceinline__ int result_row(int lane, int r) { return (lane >> 4) + 4 * r; }

// Frobenius norm squared and trace of the Hermitian matrix held in the
// result layout (every lane gets both).
__device__ __forceinline__ void norm_trace(const dbl4& cr, const dbl4& ci, int lane, double& f2, double& tr) {
  const int col = lane & 15;
  double f = 0.0, t = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    f += cr[r] * cr[r] + ci[r] * ci[r];
    if (result_row(lane, r) == col) t += cr[r];
  }
  f2 = wave_sum(f);
  tr = wave_sum(t);
}

__global__ void __launch_bounds__(256) sens_initial_kernel(const float2* __restrict__ X, int G, int ne, int64_t L,
                                                           double2* __restrict__ shat) {
  __shared__ float2 stage[kMaxSvdCoils * kEchoChunk * kStageStride];
  __shared__ double2 proj[4][16 * 16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t l0 = (int64_t)blockIdx.x * kVoxPerBlock;
  const int row_i = lane & 15, kslot = lane >> 4;

  dbl4 cr[4], ci[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    cr[v] = dbl4{0.0, 0.0, 0.0, 0.0};
    ci[v] = dbl4{0.0, 0.0, 0.0, 0.0};
  }
  // Gram matrices of the wave's four voxels, echo chunk by echo chunk
  for (int n0 = 0; n0 < ne; n0 += kEchoChunk) {
    __syncthreads();
    for (int idx = tid; idx < G * kEchoChunk * kVoxPerBlock; idx += 256) {
      const int v = idx % kVoxPerBlock, rowe = idx / kVoxPerBlock;  // rowe = coil * kEchoChunk + echo
      const int g = rowe / kEchoChunk, n = n0 + rowe % kEchoChunk;
      const int64_t l = l0 + v;
      float2 x = make_float2(0.f, 0.f);
      if (n < ne && l < L) x = X[((int64_t)g * ne + n) * L + l];
      stage[rowe * kStageStride + v] = x;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int vox = wave * 4 + v;
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        float2 y = make_float2(0.f, 0.f);
        if (row_i < G) y = stage[(row_i * kEchoChunk + 4 * kb + kslot) * kStageStride + vox];
        herm_rank4((double)y.x, (double)y.y, cr[v], ci[v]);
      }
    }
  }
  // normalise, then square until every voxel's projector has converged
  bool live[4], last[4];
  double tr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double f2;
    norm_trace(cr[v], ci[v], lane, f2, tr[v]);
    live[v] = f2 > 0.0;  // a voxel without data keeps the zero estimate
    last[v] = false;
    const double s = live[v] ? 1.0 / sqrt(f2) : 0.0;
    cr[v] *= s;
    ci[v] *= s;
    tr[v] *= s;
  }
  for (int k = 0; k < kMaxSquarings; ++k) {
    bool any = false;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (live[v] && !last[v] && tr[v] - 1.0 < kProjTol) last[v] = true;
      else if (live[v] && last[v]) live[v] = false;  // converged and squared once more
      any |= live[v];
    }
    if (!any) break;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (!live[v]) continue;
      dbl4 nr = {0.0, 0.0, 0.0, 0.0}, ni = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int r = 0; r < 4; ++r) herm_rank4(cr[v][r], -ci[v][r], nr, ni);
      double f2, t;
      norm_trace(nr, ni, lane, f2, t);
      const double s = 1.0 / sqrt(f2);
      cr[v] = nr * s;
      ci[v] = ni * s;
      tr[v] = t * s;
    }
  }
  // read u off the column of the largest diagonal entry
  double2* B = proj[wave];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t l = l0 + wave * 4 + v;
#pragma unroll
    for (int r = 0; r < 4; ++r) B[result_row(lane, r) * 16 + row_i] = make_double2(cr[v][r], ci[v][r]);
    __syncthreads();  // every wave runs this loop the same number of times
    int jm = 0;
    double dm = B[0].x;
    for (int j = 1; j < 16; ++j)
      if (B[j * 16 + j].x > dm) {
        dm = B[j * 16 + j].x;
        jm = j;
      }
    double ur = 0.0, ui = 0.0;
    if (dm > 0.0) {
      const double s = 1.0 / sqrt(dm);
      const double2 b = B[row_i * 16 + jm];
      ur = b.x * s;
      ui = b.y * s;
    }
    // coil sum over the 16 rows (lanes 0..15 hold them, as do the other groups)
    double tr_ = ur, ti = ui;
    for (int off = 8; off > 0; off >>= 1) {
      tr_ += __shfl_xor(tr_, off);
      ti += __shfl_xor(ti, off);
    }
    const double ta = hypot(tr_, ti);
    if (ta > 0.0) {
      const double cr_ = tr_ / ta, ci_ = -ti / ta;  // conj(t) / |t|
      const double vr = ur * cr_ - ui * ci_, vi = ur * ci_ + ui * cr_;
      ur = vr;
      ui = vi;
    }
    if (lane < G && l < L) shat[(int64_t)lane * L + l] = make_double2(ur, ui);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- smoothing

struct Grid3 {
  int n[3];
  int64_t s[3];
};

__device__ __forceinline__ void coords(const Grid3& g, int64_t j, int c[3]) {
  c[0] = (int)(j % g.n[0]);
  const int64_t q = j / g.n[0];
  c[1] = (int)(q % g.n[1]);
  c[2] = (int)(q / g.n[1]);
}

// Row j of A applied to a vector given by the accessor val(d, k) (its value
// at offset k along axis d from voxel j; val(0, 0) at j itself), with the
// penalty weights from the accessor wt(d, k) (k in -1, 0, 1) and the data
// weight tj.  SENS: D2 penalty, B0: D1 penalty (tj = 1).  Offsets are only
// asked for where they lie on the grid.
template <int OP, class V, class W>
__device__ __forceinline__ double apply_row(const Grid3& g, double tj, double alpha, const int c[3], V&& val,
                                            W&& wt) {
  const double v0 = val(0, 0);
  double pen = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int n = g.n[d], cd = c[d];
    if (OP == MAP_SENS) {
      if (n < 3) continue;
      const double vm1 = cd >= 1 ? val(d, -1) : 0.0;
      const double vp1 = cd <= n - 2 ? val(d, 1) : 0.0;
      if (cd >= 2) pen += wt(d, -1) * (val(d, -2) - 2.0 * vm1 + v0);
      if (cd >= 1 && cd <= n - 2) pen -= 2.0 * wt(0, 0) * (vm1 - 2.0 * v0 + vp1);
      if (cd <= n - 3) pen += wt(d, 1) * (v0 - 2.0 * vp1 + val(d, 2));
    } else {
      if (n < 2) continue;
      if (cd >= 1) pen += wt(d, -1) * (v0 - val(d, -1));
      if (cd <= n - 2) pen -= wt(0, 0) * (val(d, 1) - v0);
    }
  }
  return fma(alpha, pen, tj * v0);
}

// The same with the weights read from memory (w [L], t [L] or unused for B0).
template <int OP, class V>
__device__ __forceinline__ double apply_row_mem(const Grid3& g, const double* __restrict__ t,
                                                const double* __restrict__ w, double alpha, int64_t j, const int c[3],
                                                V&& val) {
  return apply_row<OP>(g, OP == MAP_SENS ? t[j] : 1.0, alpha, c, val,
                       [&](int d, int k) { return w[j + k * g.s[d]]; });
}

// ---- z-marching tiles: a workgroup owns a kTileX x kTileY column of the
// grid and walks it along z, holding planes z-2 .. z+2 of the vector it
// reads (with a two-voxel halo in x and y) in an LDS ring, so that each
// value is read from memory about (36 x 12) / (32 x 8) = 1.7 times instead
// of once per stencil point.
constexpr int kTileX = 32, kTileY = 8, kHalo = 2;
constexpr int kPlaneX = kTileX + 2 * kHalo, kPlaneY = kTileY + 2 * kHalo, kPlane = kPlaneX * kPlaneY;
constexpr int kRing = 2 * kHalo + 1;

__host__ __device__ __forceinline__ int tile_count(const Grid3& g) {
  return ((g.n[0] + kTileX - 1) / kTileX) * ((g.n[1] + kTileY - 1) / kTileY);
}

// load(i, interior, x, y, z): value of voxel i at (x, y, z) (interior: i
// belongs to this tile); cload(j): the per-voxel values the output of voxel
// j needs besides the stencil (right-hand side, inverse diagonal, data
// weight); row(j, c, val, wt, cv): the output of voxel j at coordinates c
// from the accessors of the vector and of the penalty weights w, whose
// planes z-1 .. z+1 are held in a second LDS ring, and cv = cload(j).  The
// vector's plane two ahead, the weights' plane one ahead and the next
// plane's per-voxel values are fetched into registers while the current
// plane is computed, so the loads of one plane overlap the arithmetic of
// the last.
constexpr int kWRing = 3;

template <class Load, class CLoad, class Row>
__device__ __forceinline__ void march(const Grid3& g, double (*ring)[kPlane], double (*wring)[kPlane],
                                      const double* __restrict__ w, Load&& load, CLoad&& cload, Row&& row) {
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int ntx = (nx + kTileX - 1) / kTileX;
  const int x0 = (int)(blockIdx.x % ntx) * kTileX, y0 = (int)(blockIdx.x / ntx) * kTileY;
  // plane entries of this thread: e0 and e1 = e0 + 256 (kPlane < 512)
  const int e0 = threadIdx.x, e1 = threadIdx.x + 256;
  const bool has1 = e1 < kPlane;
  auto at_e = [&](int e, int& gx, int& gy, bool& interior) {
    const int lx = e % kPlaneX, ly = e / kPlaneX;
    gx = x0 - kHalo + lx;
    gy = y0 - kHalo + ly;
    interior = lx >= kHalo && lx < kHalo + kTileX && ly >= kHalo && ly < kHalo + kTileY;
    return gx >= 0 && gx < nx && gy >= 0 && gy < ny;
  };
  auto fetch = [&](int z, int e) -> double {
    int gx, gy;
    bool interior;
    if (!at_e(e, gx, gy, interior)) return 0.0;
    return load(gx + g.s[1] * gy + g.s[2] * z, interior, gx, gy, z);
  };
  auto fetch_w = [&](int z, int e) -> double {
    int gx, gy;
    bool interior;
    if (!at_e(e, gx, gy, interior)) return 0.0;
    return w[gx + g.s[1] * gy + g.s[2] * z];
  };
  const int lx = threadIdx.x % kTileX, ly = threadIdx.x / kTileX;
  const int gx = x0 + lx, gy = y0 + ly;
  const bool mine = gx < nx && gy < ny;
  const int ctr = (ly + kHalo) * kPlaneX + lx + kHalo;
  for (int z = 0; z < kHalo && z < nz; ++z) {
    ring[z % kRing][e0] = fetch(z, e0);
    if (has1) ring[z % kRing][e1] = fetch(z, e1);
  }
  wring[0][e0] = fetch_w(0, e0);
  if (has1) wring[0][e1] = fetch_w(0, e1);
  double n0 = 0.0, n1 = 0.0, m0 = 0.0, m1 = 0.0;
  auto at_ij = [&](int z) { return (int64_t)gx + g.s[1] * gy + g.s[2] * z; };
  decltype(cload(int64_t(0))) cv{};
  if (mine) cv = cload(at_ij(0));
  if (kHalo < nz) {
    n0 = fetch(kHalo, e0);
    if (has1) n1 = fetch(kHalo, e1);
  }
  if (1 < nz) {
    m0 = fetch_w(1, e0);
    if (has1) m1 = fetch_w(1, e1);
  }
  for (int z = 0; z < nz; ++z) {
    if (z + kHalo < nz) {
      ring[(z + kHalo) % kRing][e0] = n0;
      if (has1) ring[(z + kHalo) % kRing][e1] = n1;
    }
    if (z + 1 < nz) {
      wring[(z + 1) % kWRing][e0] = m0;
      if (has1) wring[(z + 1) % kWRing][e1] = m1;
    }
    __syncthreads();
    if (z + kHalo + 1 < nz) {
      n0 = fetch(z + kHalo + 1, e0);
      if (has1) n1 = fetch(z + kHalo + 1, e1);
    }
    if (z + 2 < nz) {
      m0 = fetch_w(z + 2, e0);
      if (has1) m1 = fetch_w(z + 2, e1);
    }
    decltype(cv) cn{};
    if (mine && z + 1 < nz) cn = cload(at_ij(z + 1));
    if (mine) {
      const int c[3] = {gx, gy, z};
      const int64_t j = at_ij(z);
      const double* here = ring[z % kRing];
      const double* what = wring[z % kWRing];
      auto val = [&](int d, int k) -> double {
        if (d == 0) return here[ctr + k];
        if (d == 1) return here[ctr + k * kPlaneX];
        return ring[(z + k + kRing) % kRing][ctr];
      };
      auto wt = [&](int d, int k) -> double {
        if (d == 0) return what[ctr + k];
        if (d == 1) return what[ctr + k * kPlaneX];
        return wring[(z + k + kWRing) % kWRing][ctr];
      };
      row(j, c, val, wt, cv);
    }
    cv = cn;
    __syncthreads();
  }
}

template <int OP>
__device__ __forceinline__ double diag_row(const Grid3& g, const double* __restrict__ t, const double* __restrict__ w,
                                           double alpha, int64_t j, const int c[3]) {
  double pen = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int n = g.n[d], cd = c[d];
    const int64_t s = g.s[d];
    if (OP == MAP_SENS) {
      if (n < 3) continue;
      if (cd >= 2) pen += w[j - s];
      if (cd >= 1 && cd <= n - 2) pen += 4.0 * w[j];
      if (cd <= n - 3) pen += w[j + s];
    } else {
      if (n < 2) continue;
      if (cd >= 1) pen += w[j - s];
      if (cd <= n - 2) pen += w[j];
    }
  }
  const double tj = OP == MAP_SENS ? t[j] : 1.0;
  return fma(alpha, pen, tj);
}

// Sum of v over the workgroup (256 threads) in a fixed tree; valid in thread 0.
__device__ __forceinline__ double block_total(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Weights and the inverse diagonal: SENS t = mT^2, w = mR^2 (float masks);
// B0 w = eps^2 (float64 eps, t unused).
template <int OP>
__global__ void __launch_bounds__(256) smooth_setup_kernel(Grid3 g, int64_t L, const float* __restrict__ mT,
                                                           const float* __restrict__ mR,
                                                           const double* __restrict__ eps, double alpha,
                                                           double* __restrict__ t, double* __restrict__ w) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= L) return;
  if (OP == MAP_SENS) {
    const double a = mT[j], b = mR[j];
    t[j] = a * a;
    w[j] = b * b;
  } else {
    const double e = eps[j];
    w[j] = e * e;
  }
}

template <int OP>
__global__ void __launch_bounds__(256) smooth_dinv_kernel(Grid3 g, int64_t L, const double* __restrict__ t,
                                                          const double* __restrict__ w, double alpha,
                                                          double* __restrict__ dinv) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= L) return;
  int c[3];
  coords(g, j, c);
  const double d = diag_row<OP>(g, t, w, alpha, j, c);
  dinv[j] = d > 0.0 ? 1.0 / d : 0.0;
}

// Search direction at voxel i: z_i + beta p_old_i with z = D^-1 r (Jacobi)
// or the stored multigrid output (one expression for every use, so stored
// and recomputed values agree bitwise).
template <bool MG>
__device__ __forceinline__ double dir_at(const double* __restrict__ dinv, const double* __restrict__ r,
                                         const double* __restrict__ z, const double* __restrict__ po, double beta,
                                         int64_t i) {
  return MG ? fma(beta, po[i], z[i]) : fma(beta, po[i], dinv[i] * r[i]);
}

// x = 0, r = b, p = 0; partials of b.b (part1) and, for Jacobi, r.(D^-1 r)
// (part0); the status of every right-hand side cleared.
template <bool MG>
__global__ void __launch_bounds__(256) pcg_init_kernel(PcgState st, const double* __restrict__ b) {
  __shared__ double red[4];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int rhs = blockIdx.y;
  const size_t o = (size_t)rhs * st.Lp;
  double bb = 0.0, rz = 0.0;
  if (j < st.L) {
    const double bj = b[o + j];
    st.x[o + j] = 0.0;
    st.r[o + j] = bj;
    st.p[0][o + j] = 0.0;
    bb = bj * bj;
    if (!MG) rz = bj * (st.dinv[j] * bj);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st.status[rhs] = 0;
  bb = block_total(bb, red);
  if (!MG) rz = block_total(rz, red);
  if (threadIdx.x == 0) {
    st.part1[(size_t)rhs * st.npart + blockIdx.x] = bb;
    if (!MG) st.part0[(size_t)rhs * st.npart + blockIdx.x] = rz;
  }
}

__device__ __forceinline__ double sum_parts(const double* part, int nblk, double* red) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) s += part[i];
  return block_total(s, red);
}

// Single-level multigrid (the explicit inverse alone): z cleared on the
// rows of A without entries as in the last sweep below; partials of r.z
// into part0.
__global__ void __launch_bounds__(256) pcg_dot_kernel(PcgState st) {
  __shared__ double red[4];
  const int rhs = blockIdx.y;
  if (st.status[rhs]) return;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const size_t o = (size_t)rhs * st.Lp;
  double rz = 0.0;
  if (j < st.L) {
    double zj = st.z[o + j];
    if (st.dinv[j] == 0.0) {
      zj = 0.0;
      st.z[o + j] = 0.0;
    }
    rz = st.r[o + j] * zj;
  }
  rz = block_total(rz, red);
  if (threadIdx.x == 0) st.part0[(size_t)rhs * st.npart + blockIdx.x] = rz;
}

// n0: number of part0 partials (r.z from the vector or the stencil kernels)
__global__ void __launch_bounds__(256) pcg_init_scalars_kernel(PcgState st, int n0) {
  __shared__ double red[4];
  const int rhs = blockIdx.x;
  const double rz = sum_parts(st.part0 + (size_t)rhs * st.npart, n0, red);
  const double bb = sum_parts(st.part1 + (size_t)rhs * st.npart, st.nblk, red);
  if (threadIdx.x == 0) {
    st.bb[rhs] = bb;
    st.rr[rhs] = bb;
    st.rz[rhs] = rz;
    st.beta[rhs] = 0.0;
    st.alpha[rhs] = 0.0;
    st.iters[rhs] = 0;
    st.status[rhs] = bb > 0.0 ? 0 : PCG_EXACT;
  }
}

// p_new = z + beta p_old (stored), q = A p_new; partial p_new.q.  Grid
// (tiles, right-hand sides).
template <int OP, bool MG>
__global__ void __launch_bounds__(256) pcg_apply_kernel(PcgState st, Grid3 g, const double* __restrict__ t,
                                                        const double* __restrict__ w, double alpha, int pin) {
  __shared__ double ring[kRing][kPlane];
  __shared__ double wring[kWRing][kPlane];
  __shared__ double red[4];
  const int rhs = blockIdx.y;
  if (st.status[rhs]) return;  // uniform per workgroup
  const size_t o = (size_t)rhs * st.Lp;
  const double* r = st.r + o;
  const double* z = MG ? st.z + o : nullptr;
  const double* po = st.p[pin] + o;
  double* pn = st.p[pin ^ 1] + o;
  double* q = st.q + o;
  const double beta = st.beta[rhs];
  const double* dinv = st.dinv;
  double pq = 0.0;
  march(
      g, ring, wring, w,
      [&](int64_t i, bool interior, int, int, int) {
        const double v = dir_at<MG>(dinv, r, z, po, beta, i);
        if (interior) pn[i] = v;
        return v;
      },
      [&](int64_t j) { return OP == MAP_SENS ? t[j] : 1.0; },
      [&](int64_t j, const int c[3], auto& val, auto& wt, double tj) {
        const double qj = apply_row<OP>(g, tj, alpha, c, val, wt);
        q[j] = qj;
        pq += val(0, 0) * qj;
      });
  pq = block_total(pq, red);
  if (threadIdx.x == 0) st.part0[(size_t)rhs * st.npart + blockIdx.x] = pq;
}

__global__ void __launch_bounds__(256) pcg_alpha_kernel(PcgState st) {
  __shared__ double red[4];
  const int rhs = blockIdx.x;
  if (st.status[rhs]) return;
  const double pq = sum_parts(st.part0 + (size_t)rhs * st.npart, st.ntile, red);
  if (threadIdx.x == 0) {
    const double a = st.rz[rhs] / pq;
    if (!(pq > 0.0) || !isfinite(a)) {
      st.status[rhs] = PCG_BREAKDOWN;
      st.alpha[rhs] = 0.0;
    } else {
      st.alpha[rhs] = a;
    }
  }
}

// x += alpha p, r -= alpha q; partials of r.r (part1) and, for Jacobi,
// r.(D^-1 r) (part0).
template <bool MG>
__global__ void __launch_bounds__(256) pcg_update_kernel(PcgState st, int pnew) {
  __shared__ double red[4];
  const int rhs = blockIdx.y;
  if (st.status[rhs]) return;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const size_t o = (size_t)rhs * st.Lp;
  const double a = st.alpha[rhs];
  double rz = 0.0, rr = 0.0;
  if (j < st.L) {
    const double pj = st.p[pnew][o + j];
    st.x[o + j] = fma(a, pj, st.x[o + j]);
    const double rj = fma(-a, st.q[o + j], st.r[o + j]);
    st.r[o + j] = rj;
    if (!MG) rz = rj * (st.dinv[j] * rj);
    rr = rj * rj;
  }
  if (!MG) rz = block_total(rz, red);
  rr = block_total(rr, red);
  if (threadIdx.x == 0) {
    if (!MG) st.part0[(size_t)rhs * st.npart + blockIdx.x] = rz;
    st.part1[(size_t)rhs * st.npart + blockIdx.x] = rr;
  }
}

__global__ void __launch_bounds__(256) pcg_beta_kernel(PcgState st, double tol2, int n0) {
  __shared__ double red[4];
  const int rhs = blockIdx.x;
  if (st.status[rhs]) return;
  const double rz = sum_parts(st.part0 + (size_t)rhs * st.npart, n0, red);
  const double rr = sum_parts(st.part1 + (size_t)rhs * st.npart, st.nblk, red);
  if (threadIdx.x == 0) {
    st.iters[rhs] += 1;
    st.rr[rhs] = rr;
    const double bt = rz / st.rz[rhs];
    if (rr == 0.0) st.status[rhs] = PCG_EXACT;
    else if (rr <= tol2 * st.bb[rhs]) st.status[rhs] = PCG_TOL;
    else if (!isfinite(bt)) st.status[rhs] = PCG_BREAKDOWN;
    st.beta[rhs] = bt;
    st.rz[rhs] = rz;
  }
}

// ------------------------------------------------------ multigrid V-cycle
//
// Levels are rediscretisations of the same normal equations: each coarser
// grid keeps every axis of length <= 2 and halves the others (coarse point
// I at fine point 2I), its weights t, w are the interpolation-weighted
// averages of the finer ones and its penalty weight alpha is divided by 16
// (second differences) or 4 (first differences), the factor by which the
// Galerkin product P^T A P scales those terms.  Prolongation P is
// multilinear interpolation, restriction P^T divided by the constant 2^(axes
// halved), so the cycle is symmetric; smoothing is damped Jacobi (the same
// number of sweeps before and after); the coarsest level (at most
// kMgCoarseMax unknowns) is solved with its explicit inverse.

// Coarse neighbours of fine coordinate i along an axis of fine length n and
// coarse length nc (nc == n: axis not coarsened): indices n0, n1 with
// weights w0, w1 (w1 = 0 and n1 = n0 where there is one).  Fixed size, so
// that loops over them unroll into registers.
struct AxisMap {
  int n0, n1;
  double w0, w1;
};

__device__ __forceinline__ AxisMap fine_to_coarse(int i, int n, int nc) {
  AxisMap m;
  if (nc == n) {
    m.n0 = m.n1 = i;
    m.w0 = 1.0;
    m.w1 = 0.0;
  } else if ((i & 1) == 0) {
    m.n0 = m.n1 = i >> 1;
    m.w0 = 1.0;
    m.w1 = 0.0;
  } else {
    m.n0 = i >> 1;
    m.w0 = 0.5;
    const bool two = (i >> 1) + 1 < nc;
    m.n1 = two ? (i >> 1) + 1 : m.n0;
    m.w1 = two ? 0.5 : 0.0;
  }
  return m;
}

// Fine neighbours of coarse coordinate I (fine length n, coarse length nc):
// indices f[0..2] with weights wt[0..2] (0 where absent, the index then
// clamped onto the axis: the last coarse point of an even axis lies one
// past its end).
struct FineMap {
  int f[3];
  double wt[3];
};

__device__ __forceinline__ FineMap coarse_to_fine(int I, int n, int nc) {
  FineMap m;
  if (nc == n) {
    m.f[0] = m.f[1] = m.f[2] = I;
    m.wt[0] = m.wt[2] = 0.0;
    m.wt[1] = 1.0;
    return m;
  }
#pragma unroll
  for (int d = -1; d <= 1; ++d) {
    const int i = 2 * I + d;
    const bool in = i >= 0 && i < n;
    m.f[d + 1] = in ? i : (i < 0 ? 0 : n - 1);  // absent: any valid index, weight 0
    m.wt[d + 1] = in ? (d == 0 ? 1.0 : 0.5) : 0.0;
  }
  return m;
}

// sum over the coarse neighbours of fine voxel (xi, yi, zi) of weight x value
__device__ __forceinline__ double interpolate(const double* __restrict__ cv, const Grid3& gf, const Grid3& gc, int xi,
                                              int yi, int zi) {
  const AxisMap mx = fine_to_coarse(xi, gf.n[0], gc.n[0]);
  const AxisMap my = fine_to_coarse(yi, gf.n[1], gc.n[1]);
  const AxisMap mz = fine_to_coarse(zi, gf.n[2], gc.n[2]);
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int zc = a ? mz.n1 : mz.n0;
    const double wz = a ? mz.w1 : mz.w0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int yc = b ? my.n1 : my.n0;
      const double wzy = wz * (b ? my.w1 : my.w0);
      const double* line = cv + (int64_t)zc * gc.s[2] + (int64_t)yc * gc.s[1];
      s += (wzy * mx.w0) * line[mx.n0];
      s += (wzy * mx.w1) * line[mx.n1];
    }
  }
  return s;
}

// interpolation-weighted averages of the fine weights on the coarse grid
template <int OP>
__global__ void __launch_bounds__(256) mg_coarsen_kernel(Grid3 gf, Grid3 gc, int64_t Lc, const double* __restrict__ tf,
                                                         const double* __restrict__ wf, double* __restrict__ tc,
                                                         double* __restrict__ wc) {
  const int64_t J = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (J >= Lc) return;
  int C[3];
  coords(gc, J, C);
  const FineMap mx = coarse_to_fine(C[0], gf.n[0], gc.n[0]);
  const FineMap my = coarse_to_fine(C[1], gf.n[1], gc.n[1]);
  const FineMap mz = coarse_to_fine(C[2], gf.n[2], gc.n[2]);
  double st = 0.0, sw = 0.0, s = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double wgt = mz.wt[a] * my.wt[b] * mx.wt[c];
        const int64_t i = mx.f[c] + gf.s[1] * my.f[b] + gf.s[2] * mz.f[a];
        if (OP == MAP_SENS) st += wgt * tf[i];
        sw += wgt * wf[i];
        s += wgt;
      }
  if (OP == MAP_SENS) tc[J] = st / s;
  wc[J] = sw / s;
}

// Grid (tiles, right-hand sides).  MODE
//   MG_SWEEP:    y = x + omega D^-1 (b - A x), one damped Jacobi sweep;
//   MG_RESIDUAL: y = b - A x;
//   MG_PRE:      the two sweeps from x = 0: x0 = omega D^-1 b (formed while
//                loading), y = x0 + omega D^-1 (b - A x0);
//   MG_POST:     a sweep from x + P xc (the coarse correction added while
//                loading; xc on the grid gc);
//   MG_LAST:     a sweep whose result is cleared on the rows without entries
//                (voxels the system does not see, whose solution is 0;
//                prolongation would otherwise carry coarse corrections there,
//                where CG cannot remove them; clearing keeps the
//                preconditioner symmetric on the active rows), with the
//                partial b.y per workgroup into part (the finest level:
//                b = r, y = z).
enum { MG_SWEEP = 0, MG_RESIDUAL = 1, MG_PRE = 2, MG_POST = 3, MG_LAST = 4 };

template <int OP, int MODE>
__global__ void __launch_bounds__(256) mg_stencil_kernel(const int* __restrict__ status, Grid3 g, int64_t Lp,
                                                         const double* __restrict__ t, const double* __restrict__ w,
                                                         double alpha, const double* __restrict__ dinv, double omega,
                                                         const double* __restrict__ b, const double* __restrict__ x,
                                                         double* __restrict__ y, Grid3 gc, int64_t Lpc,
                                                         const double* __restrict__ xc, double* __restrict__ part,
                                                         int npart) {
  __shared__ double ring[kRing][kPlane];
  __shared__ double wring[kWRing][kPlane];
  __shared__ double red[4];
  const int rhs = blockIdx.y;
  if (status[rhs]) return;
  const size_t o = (size_t)rhs * Lp;
  const double* xv = x + o;
  const double* bv = b + o;
  const double* cv = MODE == MG_POST ? xc + (size_t)rhs * Lpc : nullptr;
  double* yv = y + o;
  double dot = 0.0;
  march(
      g, ring, wring, w,
      [&](int64_t i, bool, int xi, int yi, int zi) -> double {
        if (MODE == MG_PRE) return omega * (dinv[i] * bv[i]);
        if (MODE != MG_POST) return xv[i];
        return xv[i] + interpolate(cv, g, gc, xi, yi, zi);
      },
      [&](int64_t j) { return double3{bv[j], MODE == MG_RESIDUAL ? 0.0 : dinv[j], OP == MAP_SENS ? t[j] : 1.0}; },
      [&](int64_t j, const int c[3], auto& val, auto& wt, double3 cv) {
        const double res = cv.x - apply_row<OP>(g, cv.z, alpha, c, val, wt);
        if (MODE == MG_RESIDUAL) {
          yv[j] = res;
          return;
        }
        const double dj = cv.y;
        double yj = fma(omega, dj * res, val(0, 0));
        if (MODE == MG_LAST) {
          if (dj == 0.0) yj = 0.0;
          dot += cv.x * yj;
        }
        yv[j] = yj;
      });
  if (MODE == MG_LAST) {
    dot = block_total(dot, red);
    if (threadIdx.x == 0) part[(size_t)rhs * npart + blockIdx.x] = dot;
  }
}

// Grid of the transfer kernels: (x chunks of 64, rows y + ny z strided by
// gridDim.y, right-hand sides); one wave per workgroup, coordinates from the
// block indices.
constexpr int kRowChunk = 64;

// bc = P^T r / fac on the coarse grid
__global__ void __launch_bounds__(64) mg_restrict_kernel(const int* __restrict__ status, Grid3 gf, Grid3 gc,
                                                         int64_t Lpf, int64_t Lpc, double inv_fac,
                                                         const double* __restrict__ r, double* __restrict__ bc) {
  const int rhs = blockIdx.z;
  if (status[rhs]) return;
  const int X = blockIdx.x * kRowChunk + threadIdx.x;
  if (X >= gc.n[0]) return;
  const FineMap mx = coarse_to_fine(X, gf.n[0], gc.n[0]);
  const double* rv = r + (size_t)rhs * Lpf;
  double* bv = bc + (size_t)rhs * Lpc;
  for (int row = blockIdx.y; row < gc.n[1] * gc.n[2]; row += gridDim.y) {
    const int Y = row % gc.n[1], Z = row / gc.n[1];
    const FineMap my = coarse_to_fine(Y, gf.n[1], gc.n[1]);
    const FineMap mz = coarse_to_fine(Z, gf.n[2], gc.n[2]);
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double* line = rv + (int64_t)mz.f[a] * gf.s[2] + (int64_t)my.f[b] * gf.s[1];
        const double wzy = mz.wt[a] * my.wt[b];
#pragma unroll
        for (int c = 0; c < 3; ++c) s += (wzy * mx.wt[c]) * line[mx.f[c]];
      }
    bv[X + (int64_t)Y * gc.s[1] + (int64_t)Z * gc.s[2]] = s * inv_fac;
  }
}

// Explicit inverse of the coarsest operator (n <= kMgCoarseMax unknowns; a
// row without entries gets a unit diagonal), Gauss-Jordan in LDS.
template <int OP>
__global__ void __launch_bounds__(256) mg_coarsest_kernel(Grid3 g, int n, const double* __restrict__ t,
                                                          const double* __restrict__ w, double alpha,
                                                          double* __restrict__ ainv) {
  __shared__ double M[kMgCoarseMax][2 * kMgCoarseMax + 1];
  __shared__ double col[kMgCoarseMax];
  if (n > kMgCoarseMax) return;  // the host never builds such a hierarchy
  for (int e = threadIdx.x; e < n * n; e += 256) {
    const int i = e / n, jj = e % n;
    int c[3];
    coords(g, i, c);
    M[i][jj] = apply_row_mem<OP>(g, t, w, alpha, i, c, [&](int d, int k) { return i + k * g.s[d] == jj ? 1.0 : 0.0; });
    M[i][n + jj] = i == jj ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 256)
    if (M[i][i] == 0.0) M[i][i] = 1.0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double piv = M[k][k];
    __syncthreads();
    for (int jj = threadIdx.x; jj < 2 * n; jj += 256) M[k][jj] /= piv;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 256) col[i] = M[i][k];
    __syncthreads();
    for (int e = threadIdx.x; e < n * 2 * n; e += 256) {
      const int i = e / (2 * n), jj = e % (2 * n);
      if (i != k) M[i][jj] = fma(-col[i], M[k][jj], M[i][jj]);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < n * n; e += 256) ainv[e] = M[e / n][n + e % n];
}

__global__ void __launch_bounds__(64) mg_coarse_solve_kernel(const int* __restrict__ status, int n, int64_t Lp,
                                                             const double* __restrict__ ainv,
                                                             const double* __restrict__ b, double* __restrict__ x) {
  const int rhs = blockIdx.x;
  if (status[rhs]) return;
  const double* bv = b + (size_t)rhs * Lp;
  for (int i = threadIdx.x; i < n; i += 64) {
    double s = 0.0;
    for (int k = 0; k < n; ++k) s = fma(ainv[i * n + k], bv[k], s);
    x[(size_t)rhs * Lp + i] = s;
  }
}

// Right-hand sides of the sensitivity smoothing from S^ [G][L]:
// rows c, G + c, 2G + c = mT |S^|, mT Re(S^/|S^|), mT Im(S^/|S^|).
__global__ void __launch_bounds__(256) sens_rhs_kernel(const double2* __restrict__ shat, const float* __restrict__ mT,
                                                       int G, int64_t L, int64_t Lp, double* __restrict__ b) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (j >= L) return;
  const double2 s = shat[(int64_t)c * L + j];
  const double m = hypot(s.x, s.y);
  const double nr = m > 0.0 ? s.x / m : 0.0, ni = m > 0.0 ? s.y / m : 0.0;
  const double wt = mT[j];
  b[(size_t)c * Lp + j] = wt * m;
  b[(size_t)(G + c) * Lp + j] = wt * nr;
  b[(size_t)(2 * G + c) * Lp + j] = wt * ni;
}

// S = |S|_s n_s / |n_s| from the smoothed components.
__global__ void __launch_bounds__(256) sens_combine_kernel(const double* __restrict__ x, int G, int64_t L, int64_t Lp,
                                                           float2* __restrict__ s32, double2* __restrict__ s64) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (j >= L) return;
  const double m = x[(size_t)c * Lp + j];
  const double nr = x[(size_t)(G + c) * Lp + j], ni = x[(size_t)(2 * G + c) * Lp + j];
  const double a = hypot(nr, ni);
  double sr = 0.0, si = 0.0;
  if (a > 0.0) {
    sr = (m * nr) / a;
    si = (m * ni) / a;
  }
  if (s32) s32[(int64_t)c * L + j] = make_float2((float)sr, (float)si);
  if (s64) s64[(int64_t)c * L + j] = make_double2(sr, si);
}

// Float64 modulo with the sign of the divisor (floor modulo).
__device__ __forceinline__ double floor_mod(double a, double b) {
  double m = fmod(a, b);
  if (m != 0.0 && ((b < 0.0) != (m < 0.0))) m += b;
  return m;
}

__global__ void __launch_bounds__(256) b0_fit_kernel(const float2* __restrict__ X, const float2* __restrict__ S, int G,
                                                     int ne, int64_t L, double dte, double* __restrict__ b0hat,
                                                     double* __restrict__ beta, double* __restrict__ eps) {
  const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (l >= L) return;
  double wsum = 0.0;
  for (int g = 0; g < G; ++g) {
    const float2 s = S[(int64_t)g * L + l];
    wsum += (double)s.x * s.x + (double)s.y * s.y;
  }
  const double winv = 1.0 / (wsum > 0.0 ? wsum : 1.0);
  const double pi = 3.14159265358979311600, two_pi = 2.0 * pi;
  double c0r = 0.0, c0i = 0.0, prev = 0.0, corr = 0.0;
  double snp = 0.0, smp = 0.0, snn = 0.0, snm = 0.0, smm = 0.0;
  // first pass: unwrapped phases and the fit sums; second pass: residuals
  double phis[kMaxFitEchoes];
  for (int n = 0; n < ne; ++n) {
    double cr = 0.0, ci = 0.0;
    for (int g = 0; g < G; ++g) {
      const float2 s = S[(int64_t)g * L + l];
      const float2 x = X[((int64_t)g * ne + n) * L + l];
      const double sr = s.x, si = s.y, xr = x.x, xi = x.y;
      cr += sr * xr + si * xi;  // conj(s) x
      ci += sr * xi - si * xr;
    }
    cr *= winv;
    ci *= winv;
    if (n == 0) {
      c0r = cr;
      c0i = ci;
    }
    // phase of c_n conj(c_0)
    const double pr = cr * c0r + ci * c0i, pim = ci * c0r - cr * c0i;
    const double ph = n > 0 ? atan2(pim, pr) : 0.0;  // the first echo's phase is the reference
    double up = ph;
    if (n > 0) {
      const double dd = ph - prev;
      double dm = floor_mod(dd + pi, two_pi) - pi;
      if (dm == -pi && dd > 0.0) dm = pi;
      if (fabs(dd) >= pi) corr += dm - dd;
      up = ph + corr;
    }
    prev = ph;
    phis[n] = up;
    const double dn = n, dmn = n & 1;
    snp += dn * up;
    smp += dmn * up;
    snn += dn * dn;
    snm += dn * dmn;
    smm += dmn * dmn;
  }
  const double det = snn * smm - snm * snm;
  const double a = (smm * snp - snm * smp) / det;
  const double bcoef = (snn * smp - snm * snp) / det;
  double ss = 0.0;
  for (int n = 0; n < ne; ++n) {
    const double res = phis[n] - (a * n + bcoef * (n & 1));
    ss += res * res;
  }
  b0hat[l] = a / dte;
  beta[l] = bcoef;
  eps[l] = sqrt(ss / ne);
}

__global__ void __launch_bounds__(256) b0_store_kernel(const double* __restrict__ x, int64_t L, float* __restrict__ b0,
                                                       double* __restrict__ b064) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= L) return;
  if (b0) b0[j] = (float)x[j];
  if (b064) b064[j] = x[j];
}

Grid3 make_grid(int nx, int ny, int nz) {
  Grid3 g;
  g.n[0] = nx;
  g.n[1] = ny;
  g.n[2] = nz;
  g.s[0] = 1;
  g.s[1] = nx;
  g.s[2] = (int64_t)nx * ny;
  return g;
}

unsigned cdiv_u(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

dim3 row_grid(const Grid3& g, int nrhs) {
  const int64_t rows = (int64_t)g.n[1] * g.n[2];
  return dim3(cdiv_u(g.n[0], kRowChunk), (unsigned)std::min<int64_t>(rows, 65535), nrhs);
}

}  // namespace

size_t pcg_state_bytes(int nrhs, int nx, int ny, int nz, bool with_z) {
  const int64_t L = (int64_t)nx * ny * nz;
  const int64_t Lp = (L + 63) & ~(int64_t)63;
  const int64_t nblk = std::max<int64_t>((L + 255) / 256, tile_count(make_grid(nx, ny, nz)));
  size_t b = 0;
  auto add = [&](size_t n) { b += (n + 255) & ~(size_t)255; };
  for (int i = 0; i < (with_z ? 6 : 5); ++i) add((size_t)nrhs * Lp * 8);  // x r p0 p1 q (z)
  add((size_t)Lp * 8);                                                      // dinv
  add((size_t)nrhs * nblk * 8);                                             // part0
  add((size_t)nrhs * nblk * 8);                                             // part1
  for (int i = 0; i < 7; ++i) add((size_t)nrhs * 8);  // rz alpha beta bb rr iters status
  return b;
}

PcgState pcg_state(void* base, int nrhs, int nx, int ny, int nz, bool with_z) {
  PcgState st;
  const int64_t L = (int64_t)nx * ny * nz;
  st.L = L;
  st.Lp = (L + 63) & ~(int64_t)63;
  st.nblk = (int)((L + 255) / 256);
  st.ntile = tile_count(make_grid(nx, ny, nz));
  st.npart = std::max(st.nblk, st.ntile);
  st.nrhs = nrhs;
  char* p = static_cast<char*>(base);
  auto take = [&](size_t n) {
    char* q = p;
    p += (n + 255) & ~(size_t)255;
    return q;
  };
  const size_t vec = (size_t)nrhs * st.Lp * 8;
  st.x = (double*)take(vec);
  st.r = (double*)take(vec);
  st.p[0] = (double*)take(vec);
  st.p[1] = (double*)take(vec);
  st.q = (double*)take(vec);
  st.z = with_z ? (double*)take(vec) : nullptr;
  st.dinv = (double*)take((size_t)st.Lp * 8);
  st.part0 = (double*)take((size_t)nrhs * st.npart * 8);
  st.part1 = (double*)take((size_t)nrhs * st.npart * 8);
  st.rz = (double*)take((size_t)nrhs * 8);
  st.alpha = (double*)take((size_t)nrhs * 8);
  st.beta = (double*)take((size_t)nrhs * 8);
  st.bb = (double*)take((size_t)nrhs * 8);
  st.rr = (double*)take((size_t)nrhs * 8);
  st.iters = (int*)take((size_t)nrhs * 8);
  st.status = (int*)take((size_t)nrhs * 8);
  return st;
}

namespace {

constexpr int kMgMaxLevels = 24;
constexpr double kMgOmega = 0.6;  // damped Jacobi weight
constexpr int kMgSweeps = 2;      // sweeps before and after the coarse correction

struct MgLevel {
  Grid3 g;
  int64_t L, Lp;
  double alpha;
  const double* t;
  const double* w;
  const double* dinv;
  const double* b;
  double* x[2];
  double* tw[3];  // coarse levels: t, w, dinv storage
};

struct MgHierarchy {
  int nlev = 0;
  MgLevel lev[kMgMaxLevels];
  double* ainv = nullptr;
};

// Grid sizes of the levels (fine first).
int mg_dims(int nx, int ny, int nz, int dims[][3]) {
  int n = 0;
  int d[3] = {nx, ny, nz};
  for (;;) {
    dims[n][0] = d[0];
    dims[n][1] = d[1];
    dims[n][2] = d[2];
    ++n;
    const int64_t L = (int64_t)d[0] * d[1] * d[2];
    if (L <= kMgCoarseMax || n == kMgMaxLevels) break;
    int c[3];
    for (int k = 0; k < 3; ++k) c[k] = d[k] >= 3 ? d[k] / 2 + 1 : d[k];
    if (c[0] == d[0] && c[1] == d[1] && c[2] == d[2]) break;
    for (int k = 0; k < 3; ++k) d[k] = c[k];
  }
  return n;
}

size_t mg_layout(void* base, int nrhs, int nx, int ny, int nz, MgHierarchy* h) {
  int dims[kMgMaxLevels][3];
  const int nlev = mg_dims(nx, ny, nz, dims);
  char* p = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t n) {
    char* q = p ? p + off : nullptr;
    off += (n + 255) & ~(size_t)255;
    return (double*)q;
  };
  if (h) h->nlev = nlev;
  for (int l = 0; l < nlev; ++l) {
    const int64_t L = (int64_t)dims[l][0] * dims[l][1] * dims[l][2];
    const int64_t Lp = (L + 63) & ~(int64_t)63;
    MgLevel lv{};
    lv.g = make_grid(dims[l][0], dims[l][1], dims[l][2]);
    lv.L = L;
    lv.Lp = Lp;
    if (l == 0) {
      lv.x[1] = take((size_t)nrhs * Lp * 8);
    } else {
      for (int k = 0; k < 3; ++k) lv.tw[k] = take((size_t)Lp * 8);
      lv.b = take((size_t)nrhs * Lp * 8);
      lv.x[0] = take((size_t)nrhs * Lp * 8);
      lv.x[1] = take((size_t)nrhs * Lp * 8);
    }
    if (h) h->lev[l] = lv;
  }
  double* ainv = take((size_t)kMgCoarseMax * kMgCoarseMax * 8);
  if (h) h->ainv = ainv;
  return off;
}

// Coarse weights, inverse diagonals and the coarsest inverse.
template <int OP>
hipError_t mg_setup(MgHierarchy& h, const PcgState& st, const double* t, const double* w, double alpha,
                    hipStream_t s) {
  const double shrink = OP == MAP_SENS ? 1.0 / 16.0 : 1.0 / 4.0;
  MgLevel& f = h.lev[0];
  f.alpha = alpha;
  f.t = t;
  f.w = w;
  f.dinv = st.dinv;
  f.b = st.r;
  f.x[0] = st.z;
  for (int l = 1; l < h.nlev; ++l) {
    MgLevel& c = h.lev[l];
    const MgLevel& p = h.lev[l - 1];
    c.alpha = p.alpha * shrink;
    c.t = c.tw[0];
    c.w = c.tw[1];
    c.dinv = c.tw[2];
    hipLaunchKernelGGL(mg_coarsen_kernel<OP>, dim3(cdiv_u(c.L, 256)), dim3(256), 0, s, p.g, c.g, c.L, p.t, p.w,
                       c.tw[0], c.tw[1]);
    hipLaunchKernelGGL(smooth_dinv_kernel<OP>, dim3(cdiv_u(c.L, 256)), dim3(256), 0, s, c.g, c.L, c.t, c.w, c.alpha,
                       c.tw[2]);
  }
  const MgLevel& z = h.lev[h.nlev - 1];
  hipLaunchKernelGGL(mg_coarsest_kernel<OP>, dim3(1), dim3(256), 0, s, z.g, (int)z.L, z.t, z.w, z.alpha, h.ainv);
  return hipGetLastError();
}

// z = M^-1 r (one V-cycle for every running right-hand side): per level the
// two pre-sweeps in one pass, the residual, its restriction; the coarsest
// solve; per level the prolongation inside the first post-sweep and the
// second post-sweep (on the finest level also clearing the rows without
// entries and forming r.z).  Every level ends in x[0] (st.z on the finest).
static_assert(kMgSweeps == 2, "the fused passes are two sweeps before and after");
template <int OP>
hipError_t mg_vcycle(const MgHierarchy& h, const PcgState& st, hipStream_t s) {
  const int nr = st.nrhs;
  for (int l = 0; l + 1 < h.nlev; ++l) {
    const MgLevel& v = h.lev[l];
    const MgLevel& n = h.lev[l + 1];
    const dim3 tg(tile_count(v.g), nr);
    hipLaunchKernelGGL((mg_stencil_kernel<OP, MG_PRE>), tg, dim3(256), 0, s, st.status, v.g, v.Lp, v.t, v.w, v.alpha,
                       v.dinv, kMgOmega, v.b, v.x[0], v.x[0], n.g, n.Lp, nullptr, nullptr, 0);
    hipLaunchKernelGGL((mg_stencil_kernel<OP, MG_RESIDUAL>), tg, dim3(256), 0, s, st.status, v.g, v.Lp, v.t, v.w,
                       v.alpha, v.dinv, kMgOmega, v.b, v.x[0], v.x[1], n.g, n.Lp, nullptr, nullptr, 0);
    double fac = 1.0;
    for (int d = 0; d < 3; ++d) fac *= n.g.n[d] != v.g.n[d] ? 2.0 : 1.0;
    hipLaunchKernelGGL(mg_restrict_kernel, row_grid(n.g, nr), dim3(kRowChunk), 0, s, st.status, v.g, n.g, v.Lp, n.Lp,
                       1.0 / fac, v.x[1], const_cast<double*>(n.b));
  }
  const MgLevel& z = h.lev[h.nlev - 1];
  hipLaunchKernelGGL(mg_coarse_solve_kernel, dim3(nr), dim3(64), 0, s, st.status, (int)z.L, z.Lp, h.ainv, z.b,
                     z.x[0]);
  for (int l = h.nlev - 2; l >= 0; --l) {
    const MgLevel& v = h.lev[l];
    const MgLevel& n = h.lev[l + 1];
    const dim3 tg(tile_count(v.g), nr);
    hipLaunchKernelGGL((mg_stencil_kernel<OP, MG_POST>), tg, dim3(256), 0, s, st.status, v.g, v.Lp, v.t, v.w, v.alpha,
                       v.dinv, kMgOmega, v.b, v.x[0], v.x[1], n.g, n.Lp, n.x[0], nullptr, 0);
    if (l > 0)
      hipLaunchKernelGGL((mg_stencil_kernel<OP, MG_SWEEP>), tg, dim3(256), 0, s, st.status, v.g, v.Lp, v.t, v.w,
                         v.alpha, v.dinv, kMgOmega, v.b, v.x[1], v.x[0], n.g, n.Lp, nullptr, nullptr, 0);
    else
      hipLaunchKernelGGL((mg_stencil_kernel<OP, MG_LAST>), tg, dim3(256), 0, s, st.status, v.g, v.Lp, v.t, v.w,
                         v.alpha, v.dinv, kMgOmega, v.b, v.x[1], v.x[0], n.g, n.Lp, nullptr, st.part0, st.npart);
  }
  return hipGetLastError();
}

template <int OP>
hipError_t pcg_run(int precond, const PcgState& st, void* mg_ws, const double* b, int nx, int ny, int nz,
                   const double* t, const double* w, double alpha, double tol, int max_iter, int* status, int* iters,
                   hipStream_t s) {
  const bool mg = precond == NFS_PRECOND_MG;
  const Grid3 g = make_grid(nx, ny, nz);
  const dim3 grid(st.nblk, st.nrhs), tgrid(st.ntile, st.nrhs);
  MgHierarchy h;
  hipError_t e;
  if (mg) {
    mg_layout(mg_ws, st.nrhs, nx, ny, nz, &h);
    if (h.lev[h.nlev - 1].L > kMgCoarseMax) return hipErrorInvalidValue;
    if ((e = mg_setup<OP>(h, st, t, w, alpha, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(pcg_init_kernel<true>, grid, dim3(256), 0, s, st, b);
    if ((e = mg_vcycle<OP>(h, st, s)) != hipSuccess) return e;
    if (h.nlev == 1) hipLaunchKernelGGL(pcg_dot_kernel, grid, dim3(256), 0, s, st);
  } else {
    hipLaunchKernelGGL(pcg_init_kernel<false>, grid, dim3(256), 0, s, st, b);
  }
  // part0 holds r.z from the vector kernels (nblk) or the last sweep (ntile)
  const int n0 = mg && h.nlev > 1 ? st.ntile : st.nblk;
  hipLaunchKernelGGL(pcg_init_scalars_kernel, dim3(st.nrhs), dim3(256), 0, s, st, n0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const double tol2 = tol * tol;
  int it = 0;
  for (;;) {
    if ((e = hipMemcpyAsync(status, st.status, st.nrhs * sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    bool all = true;
    for (int k = 0; k < st.nrhs; ++k) all = all && status[k] != 0;
    if (all || it >= max_iter) break;
    const int n = std::min(kPcgChunk, max_iter - it);
    for (int k = 0; k < n; ++k, ++it) {
      const int pin = it & 1;
      if (mg) {
        hipLaunchKernelGGL((pcg_apply_kernel<OP, true>), tgrid, dim3(256), 0, s, st, g, t, w, alpha, pin);
        hipLaunchKernelGGL(pcg_alpha_kernel, dim3(st.nrhs), dim3(256), 0, s, st);
        hipLaunchKernelGGL(pcg_update_kernel<true>, grid, dim3(256), 0, s, st, pin ^ 1);
        if ((e = mg_vcycle<OP>(h, st, s)) != hipSuccess) return e;
        if (h.nlev == 1) hipLaunchKernelGGL(pcg_dot_kernel, grid, dim3(256), 0, s, st);
      } else {
        hipLaunchKernelGGL((pcg_apply_kernel<OP, false>), tgrid, dim3(256), 0, s, st, g, t, w, alpha, pin);
        hipLaunchKernelGGL(pcg_alpha_kernel, dim3(st.nrhs), dim3(256), 0, s, st);
        hipLaunchKernelGGL(pcg_update_kernel<false>, grid, dim3(256), 0, s, st, pin ^ 1);
      }
      hipLaunchKernelGGL(pcg_beta_kernel, dim3(st.nrhs), dim3(256), 0, s, st, tol2, n0);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipMemcpy(iters, st.iters, st.nrhs * sizeof(int), hipMemcpyDeviceToHost);
}

}  // namespace

size_t mg_bytes(int nrhs, int nx, int ny, int nz) { return mg_layout(nullptr, nrhs, nx, ny, nz, nullptr); }

hipError_t pcg_solve(int op, int precond, const PcgState& st, void* mg_ws, const double* b, int nx, int ny, int nz,
                     const double* t, const double* w, double alpha, double tol, int max_iter, int* status,
                     int* iters, hipStream_t s) {
  if (st.L == 0 || st.nrhs == 0) {
    for (int k = 0; k < st.nrhs; ++k) {
      status[k] = PCG_EXACT;
      iters[k] = 0;
    }
    return hipSuccess;
  }
  return op == MAP_SENS ? pcg_run<MAP_SENS>(precond, st, mg_ws, b, nx, ny, nz, t, w, alpha, tol, max_iter, status,
                                            iters, s)
                        : pcg_run<MAP_B0>(precond, st, mg_ws, b, nx, ny, nz, t, w, alpha, tol, max_iter, status,
                                          iters, s);
}

hipError_t launch_sens_initial(const float2* X, int G, int ne, int64_t L, double2* shat, hipStream_t s) {
  if (L == 0) return hipSuccess;
  hipLaunchKernelGGL(sens_initial_kernel, dim3(cdiv_u(L, kVoxPerBlock)), dim3(256), 0, s, X, G, ne, L, shat);
  return hipGetLastError();
}

hipError_t launch_sens_rhs(const double2* shat, const float* mT, int G, int64_t L, int64_t Lp, double* b,
                           hipStream_t s) {
  if (L == 0) return hipSuccess;
  hipLaunchKernelGGL(sens_rhs_kernel, dim3(cdiv_u(L, 256), G), dim3(256), 0, s, shat, mT, G, L, Lp, b);
  return hipGetLastError();
}

hipError_t launch_sens_combine(const double* x, int G, int64_t L, int64_t Lp, float2* s32, double2* s64,
                               hipStream_t s) {
  if (L == 0) return hipSuccess;
  hipLaunchKernelGGL(sens_combine_kernel, dim3(cdiv_u(L, 256), G), dim3(256), 0, s, x, G, L, Lp, s32, s64);
  return hipGetLastError();
}

hipError_t launch_b0_fit(const float2* X, const float2* S, int G, int ne, int64_t L, double dte, double* b0hat,
                         double* beta, double* eps, hipStream_t s) {
  if (L == 0) return hipSuccess;
  hipLaunchKernelGGL(b0_fit_kernel, dim3(cdiv_u(L, 256)), dim3(256), 0, s, X, S, G, ne, L, dte, b0hat, beta, eps);
  return hipGetLastError();
}

hipError_t launch_b0_store(const double* x, int64_t L, float* b0, double* b064, hipStream_t s) {
  if (L == 0) return hipSuccess;
  hipLaunchKernelGGL(b0_store_kernel, dim3(cdiv_u(L, 256)), dim3(256), 0, s, x, L, b0, b064);
  return hipGetLastError();
}

hipError_t launch_smooth_setup(int op, int nx, int ny, int nz, const float* mT, const float* mR, const double* eps,
                               double alpha, double* t, double* w, const PcgState& st, hipStream_t s) {
  const Grid3 g = make_grid(nx, ny, nz);
  const int64_t L = st.L;
  if (L == 0) return hipSuccess;
  const dim3 grid(cdiv_u(L, 256));
  if (op == MAP_SENS) {
    hipLaunchKernelGGL(smooth_setup_kernel<MAP_SENS>, grid, dim3(256), 0, s, g, L, mT, mR, eps, alpha, t, w);
    hipLaunchKernelGGL(smooth_dinv_kernel<MAP_SENS>, grid, dim3(256), 0, s, g, L, t, w, alpha, st.dinv);
  } else {
    hipLaunchKernelGGL(smooth_setup_kernel<MAP_B0>, grid, dim3(256), 0, s, g, L, mT, mR, eps, alpha, t, w);
    hipLaunchKernelGGL(smooth_dinv_kernel<MAP_B0>, grid, dim3(256), 0, s, g, L, t, w, alpha, st.dinv);
  }
  return hipGetLastError();
}

}  // namespace nfs
