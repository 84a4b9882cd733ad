// Encoding-operator kernels for gfx950: E and E^H of higher-order SENSE.
//
// The operator (signal-model equations of the paper's Methods section,
// "Implementation of the higher-order SENSE reconstruction"):
//   phi(k, l) = sum_b kcoef[k][b] fields[b][l] + t[k] b0[l]
//   E:   y[k][c] = sum_l exp(+i phi(k, l)) Q[l][c],  Q = S o (rho 1^T)
//   E^H: Q'[l][c] = sum_k exp(-i phi(k, l)) m[c][k];  x[l] = sum_c conj(S[c][l]) Q'[l][c]
// The entries of P = exp(i phi) are never stored: every 16 x 16 block of P
// is built in registers right before the matrix cores consume it (the
// paper's split form computes blocks P' of P and applies them; here a block
// is one MFMA tile).
//
// Complex products become real ones: the generated operand of a tile is the
// row of (cos, sin) pairs, and the data operand of each streamed item is
// expanded once into a 2 x 2G real block, so that
//   E:   [y_re y_im] = [cos sin] . [[Q_re, Q_im], [-Q_im, Q_re]]
//   E^H: [x_re x_im] = [cos sin] . [[m_re, m_im], [ m_im, -m_re]]
// (real columns interleaved per coil: column 2c is re, 2c+1 is im).
#include <algorithm>

#include "nfs_internal.h"

namespace nfs {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef b8 b8_t;
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr double kInv2Pi = 0.159154943091895335768883763372514362;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---------------------------------------------------------------------------
// Phase coefficients, split into f16 parts, in MFMA fragment order.
//
// phi(k, l) = sum_b a_b(k) h_b(l) with a the sample-side coefficients
// (a_0 = t / 2 pi, a_{b+1} = kcoef[.][b] / 2 pi: phase in revolutions) and h
// the voxel-side ones (h_0 = b0, h_{b+1} = fields[b][.]).
//
// Per term, a power of two 2^e_b moves magnitude from one side to the other
// (a_b 2^-e_b and h_b 2^e_b), chosen from the two largest magnitudes so that
// both sides peak near sqrt(max|a_b| max|h_b|), inside float16's range.  Each
// balanced coefficient x (in double, so neither scaling rounds) is split as
// x1 = f16(x), x2 = f16(x - x1), x = x1 + x2 + O(2^-22 x), and the term is
// a1 h1 + a1 h2 + a2 h1: products of f16 values are exact in the float32
// accumulator of v_mfma_f32_16x16x32_f16, and the dropped a2 h2 and the
// split remainders are O(2^-21) of max|a_b| max|h_b|.
//
// K-slot layout of one 16-item chunk: 3T slots over NQ = ceil(3T / 32)
// instructions; slot b holds the (1,2) product of term b, slot T + b the
// (2,1) product and slot 2T + b the (1,1) product; slots past 3T are zero.
// The small products thus enter the running sum before the large ones.
// Slot k multiplies slot k of the other operand, so the two operands carry
// complementary parts: role A (the streamed side, MFMA operand A) takes
// part i of product (i, j), role B (the held side, operand B) part j.
// Per lane (g = lane / 16, n = lane % 16): item 16 chunk + n, slots
// 32 q + 8 g + e, e = 0..7, stored as one 16-byte vector
// out[(chunk * NQ + q) * 64 + lane].

// e_b of the balancing power for term b, from the term maxima (identical on
// both sides and in every kernel that reads it)
__device__ __forceinline__ int term_shift(const unsigned* __restrict__ tmax, int b) {
  const float ma = __uint_as_float(tmax[b]) * (float)kInv2Pi;
  const float mh = __uint_as_float(tmax[kMaxTerms + b]);
  if (!(ma > 0.f) || !(mh > 0.f) || !isfinite(ma) || !isfinite(mh)) return 0;
  int ea, eh;
  frexpf(ma, &ea);
  frexpf(mh, &eh);
  return (ea - eh) / 2;
}

// largest |a_b| (side 0, before the 1/2pi scaling) and |h_b| (side 1) per
// term; grid (kTmaxBlocks, 2), one atomic max per term per workgroup
__global__ __launch_bounds__(256) void term_absmax_kernel(const float* __restrict__ t, const float* __restrict__ kcoef,
                                                          int64_t K, const float* __restrict__ b0,
                                                          const float* __restrict__ fields, int64_t L, int P,
                                                          unsigned* __restrict__ tmax) {
  const int side = blockIdx.y;
  const int64_t n = side == 0 ? K : L;
  const float* c0 = side == 0 ? t : b0;
  float mx[kMaxTerms];
#pragma unroll
  for (int b = 0; b < kMaxTerms; ++b) mx[b] = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    mx[0] = fmaxf(mx[0], fabsf(c0[i]));
#pragma unroll
    for (int b = 1; b < kMaxTerms; ++b)
      if (b <= P) {
        const float v = side == 0 ? kcoef[i * P + (b - 1)] : fields[(int64_t)(b - 1) * L + i];
        mx[b] = fmaxf(mx[b], fabsf(v));
      }
  }
  __shared__ float red[kWaves][kMaxTerms];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int b = 0; b < kMaxTerms; ++b) {
    float v = mx[b];
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    if (lane == 0) red[wave][b] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x <= P) {
    float v = red[0][threadIdx.x];
    for (int w = 1; w < kWaves; ++w) v = fmaxf(v, red[w][threadIdx.x]);
    if (v > 0.f) atomicMax(&tmax[side * kMaxTerms + threadIdx.x], __float_as_uint(v));
  }
}

// side 0: samples (t, kcoef, K items); side 1: voxels (b0, fields, L items)
__global__ void pack_phase_kernel(const float* __restrict__ c0, const float* __restrict__ cb, int64_t n_items,
                                  int P, int side, int role, int NQ, const unsigned* __restrict__ tmax,
                                  h8* __restrict__ out, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int lane = (int)(i & 63);
  const int64_t qq = i >> 6;
  const int q = (int)(qq % NQ);
  const int64_t chunk = qq / NQ;
  const int64_t item = chunk * kChunk + (lane & 15);
  const int g = lane >> 4;
  const int T = P + 1;
  h8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = 32 * q + 8 * g + e;
    const int pair = k / T, b = k - pair * T;
    float x = 0.f;
    if (pair < 3 && item < n_items) {
      // part of this side in product `pair`: (1,2), (2,1), (1,1)
      const int part = pair == 2 ? 1 : ((pair == 0) == (role == 0) ? 1 : 2);
      const int sh = term_shift(tmax, b);
      double c;
      if (side == 0)
        c = ldexp((b == 0 ? (double)c0[item] : (double)cb[item * P + (b - 1)]) * kInv2Pi, -sh);
      else
        c = ldexp(b == 0 ? (double)c0[item] : (double)cb[(int64_t)(b - 1) * n_items + item], sh);
      const float x1 = (float)(_Float16)(float)c;
      x = part == 1 ? x1 : (float)(_Float16)(float)(c - (double)x1);
    }
    v[e] = (_Float16)x;
  }
  out[i] = v;
}

__global__ void scale_sens_kernel(const float2* __restrict__ sens, const float* __restrict__ icorr, int G,
                                  int64_t L, float2* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)G * L) return;
  const float j = icorr[i % L];
  const float2 s = sens[i];
  out[i] = make_float2(s.x * j, s.y * j);
}

// ---------------------------------------------------------------------------
// Largest |re| or |im| of value(item, c) = src[item*is + c*cs] * mul[c][item] * wgt[item]
// per workgroup (kBmaxBlocks workgroups, every entry of bmax written).
__global__ __launch_bounds__(256) void absmax_kernel(const float2* __restrict__ src,
                                                     const float2* __restrict__ mul, const float* __restrict__ wgt,
                                                     int64_t n_items, int64_t is, int64_t cs, int G,
                                                     float* __restrict__ bmax, const int* stop) {
  if (stop && *stop) return;
  __shared__ float red[256];
  float mx = 0.f;
  for (int64_t item = (int64_t)blockIdx.x * 256 + threadIdx.x; item < n_items;
       item += (int64_t)gridDim.x * 256) {
    const float w = wgt ? fabsf(wgt[item]) : 1.f;
    for (int c = 0; c < G; ++c) {
      float2 v = src[item * is + (int64_t)c * cs];
      if (mul) v = cmul(mul[(int64_t)c * n_items + item], v);
      mx = fmaxf(mx, w * fmaxf(fabsf(v.x), fabsf(v.y)));
    }
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) bmax[blockIdx.x] = red[0];
}

// One lane's 8 fragment values of (chunk ch, column block nb) in the layout
// of precision PREC (see below).
template <int PREC>
__device__ __forceinline__ void store_fragment(const float (&vals)[8], void* __restrict__ out, int64_t ch, int nb,
                                               int NB, int lane) {
  if (PREC == PREC_FP32) {
    h8 hi, lo;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      hi[u] = (_Float16)vals[u];
      lo[u] = (_Float16)(vals[u] - (float)hi[u]);
    }
    ((h8*)out)[((ch * NB + nb) * 2 + 0) * 64 + lane] = hi;
    ((h8*)out)[((ch * NB + nb) * 2 + 1) * 64 + lane] = lo;
  } else if (PREC == PREC_FP16) {
    h8 h;
#pragma unroll
    for (int u = 0; u < 8; ++u) h[u] = (_Float16)vals[u];
    ((h8*)out)[(ch * NB + nb) * 64 + lane] = h;
  } else {
    b8 hi, lo;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      hi[u] = (__bf16)vals[u];
      lo[u] = (__bf16)(vals[u] - (float)hi[u]);
    }
    ((b8*)out)[((ch * NB + nb) * 2 + 0) * 64 + lane] = hi;
    ((b8*)out)[((ch * NB + nb) * 2 + 1) * 64 + lane] = lo;
  }
}

// ---------------------------------------------------------------------------
// Data operand in MFMA fragment order (B side of the complex contraction).
// For chunk ch, column block nb and lane (g = lane / 16, n = lane % 16) the
// fragment holds, in slot u = 0..7, the entry for streamed item 4g + u/2,
// component u % 2 (0: the cos row, 1: the sin row) and real column
// N = 16 nb + n (coil N / 2, re/im N % 2).
//   fp16: one 16-byte vector per (ch, nb, lane): [(ch*NB + nb)*64 + lane]
//   bf16: two, the bf16 rounding v_hi of each value and v_lo = bf16(v - v_hi):
//         [((ch*NB + nb)*2 + part)*64 + lane]; the kernel runs one MFMA per
//         part into the same accumulator, so the data operand carries ~16
//         significant bits and only the (cos, sin) operand is 8-bit
//   fp32: two f16 fragments, v_hi = f16(v) and v_lo = f16(v - v_hi):
//         [((ch*NB + nb)*2 + part)*64 + lane]; v = v_hi + v_lo + O(2^-22 v)
// FP16 and FP32: the values are scaled by a power of two so that the largest
// magnitude lands just below 2^14; 1/scale is stored in *unscale.
// An optional real per-item weight wgt multiplies every value (used by the
// backward pass: t o G for the B0 gradient, h_b o rho for the field terms).
// bx: the workgroup's index in the single-slice grid (its blockIdx.x).
template <int PREC, int OP>
__device__ __forceinline__ void pack_data_body(const float2* __restrict__ src, const float2* __restrict__ mul,
                                               const float* __restrict__ wgt, int64_t n_items, int64_t is, int64_t cs,
                                               int G, int NB, int64_t nchunks, void* __restrict__ out,
                                               const float* __restrict__ bmax, float* __restrict__ unscale,
                                               const int* stop, int64_t bx) {
  if (stop && *stop) return;
  float scale = 1.f;
  if (PREC != PREC_BF16) {
    __shared__ float red[kBmaxBlocks];
    red[threadIdx.x] = bmax[threadIdx.x];
    __syncthreads();
    for (int w = kBmaxBlocks / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
      __syncthreads();
    }
    const float mx = red[0];
    if (mx > 0.f && isfinite(mx)) {
      int e;
      frexpf(mx, &e);  // mx < 2^e
      int sh = 14 - e;
      sh = sh > 100 ? 100 : (sh < -100 ? -100 : sh);
      scale = ldexpf(1.f, sh);
    }
    if (bx == 0 && threadIdx.x == 0) *unscale = 1.f / scale;
  }
  const int64_t i = bx * 256 + threadIdx.x;
  if (i >= nchunks * NB * 64) return;
  const int lane = (int)(i & 63);
  const int64_t q = i >> 6;
  const int nb = (int)(q % NB);
  const int64_t ch = q / NB;
  const int g = lane >> 4, n = lane & 15;
  const int N = nb * 16 + n;
  const int c = N >> 1, reim = N & 1;
  float vals[8];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t item = ch * kChunk + g * 4 + j;
    float2 v = make_float2(0.f, 0.f);
    if (item < n_items && c < G) {
      v = src[item * is + (int64_t)c * cs];
      if (mul) v = cmul(mul[(int64_t)c * n_items + item], v);
      const float w = wgt ? wgt[item] * scale : scale;
      v.x *= w;
      v.y *= w;
    }
    float cosrow, sinrow;
    if (OP == OP_E) {
      cosrow = reim ? v.y : v.x;
      sinrow = reim ? v.x : -v.y;
    } else {
      cosrow = reim ? v.y : v.x;
      sinrow = reim ? -v.x : v.y;
    }
    vals[2 * j] = cosrow;
    vals[2 * j + 1] = sinrow;
  }
  store_fragment<PREC>(vals, out, ch, nb, NB, lane);
}

template <int PREC, int OP>
__global__ __launch_bounds__(256) void pack_data_kernel(
    const float2* __restrict__ src, const float2* __restrict__ mul, const float* __restrict__ wgt, int64_t n_items,
    int64_t is, int64_t cs, int G, int NB, int64_t nchunks, void* __restrict__ out, const float* __restrict__ bmax,
    float* __restrict__ unscale, const int* stop) {
  pack_data_body<PREC, OP>(src, mul, wgt, n_items, is, cs, G, NB, nchunks, out, bmax, unscale, stop, blockIdx.x);
}

// The E-operand packing of the lock-step batched solve: slice blockIdx.y of
// sl, workgroups past that slice's own grid return at once.
template <int PREC>
__global__ __launch_bounds__(256) void pack_data_E_batched_kernel(const PackSlice* __restrict__ sl) {
  const PackSlice a = sl[blockIdx.y];
  if ((int64_t)blockIdx.x * 256 >= a.nchunks * a.NB * 64) return;
  pack_data_body<PREC, OP_E>((const float2*)a.src, a.mul, a.wgt, a.n_items, a.is, a.cs, a.G, a.NB, a.nchunks, a.out,
                             a.bmax, a.unscale, a.stop, blockIdx.x);
}

// E^H data operand straight from the E partials (the E^H E chain): the
// streamed items are the samples, with value(k, c) = sum over splits, in
// split order, of epart[s][k][2c] + i epart[s][k][2c + 1], times `scale`.
// FP16 and FP32: the E operand entries are below 2^14 in magnitude, so every real
// column of the E output is below 2^15 L; the caller passes scale =
// 2^-(ceil(log2 L) + 1), which keeps the packed values below 2^14 without a
// pass over the E output, and *unscale_out = *unscale_in / scale.  (Values
// far below the bound only leave float16's normal range 29 binades under
// it.)
// An optional real weight per sample, times wmul, multiplies the E output
// first (|weight * wmul| <= 1 keeps the scale bound).
template <int PREC>
__device__ __forceinline__ void pack_EH_from_epart_body(const float* __restrict__ epart, int nsplit, int64_t HC16,
                                                        int NB, int64_t K, int G, float scale,
                                                        const float* __restrict__ wgt, float wmul,
                                                        const float* __restrict__ unscale_in,
                                                        float* __restrict__ unscale_out, int64_t nchunks,
                                                        void* __restrict__ out, const int* stop, int64_t bx) {
  if (stop && *stop) return;
  if (PREC != PREC_BF16 && bx == 0 && threadIdx.x == 0) *unscale_out = *unscale_in / scale;
  const int64_t i = bx * 256 + threadIdx.x;
  if (i >= nchunks * NB * 64) return;
  const int lane = (int)(i & 63);
  const int64_t q = i >> 6;
  const int nb = (int)(q % NB);
  const int64_t ch = q / NB;
  const int g = lane >> 4, n = lane & 15;
  const int N = nb * 16 + n;
  const int c = N >> 1, reim = N & 1;
  const int64_t ncol = (int64_t)NB * 16, pstride = HC16 * ncol;
  // the four items' split sums advance together, four splits at a time, so
  // that sixteen loads are in flight; each sum is added in split order
  const float2* src[4];
  bool ok[4];
  float2 v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t item = ch * kChunk + g * 4 + j;
    ok[j] = item < K && c < G;
    src[j] = (const float2*)(epart + (ok[j] ? item : 0) * ncol + 2 * (ok[j] ? c : 0));
    v[j] = make_float2(0.f, 0.f);
  }
  const int64_t st2 = pstride / 2;
  for (int s0 = 0; s0 < nsplit; s0 += 4) {
    float2 w[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        w[j][k] = ok[j] && s0 + k < nsplit ? src[j][(int64_t)(s0 + k) * st2] : make_float2(0.f, 0.f);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (ok[j] && s0 + k < nsplit) {
          v[j].x += w[j][k].x;
          v[j].y += w[j][k].y;
        }
  }
  float vals[8];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (ok[j]) {
      const int64_t item = ch * kChunk + g * 4 + j;
      const float w = wgt ? wgt[item] * wmul : wmul;
      v[j].x *= scale * w;
      v[j].y *= scale * w;
    }
    vals[2 * j] = reim ? v[j].y : v[j].x;
    vals[2 * j + 1] = reim ? -v[j].x : v[j].y;
  }
  store_fragment<PREC>(vals, out, ch, nb, NB, lane);
}

template <int PREC>
__global__ __launch_bounds__(256) void pack_EH_from_epart_kernel(const float* __restrict__ epart, int nsplit,
                                                                 int64_t HC16, int NB, int64_t K, int G, float scale,
                                                                 const float* __restrict__ wgt, float wmul,
                                                                 const float* __restrict__ unscale_in,
                                                                 float* __restrict__ unscale_out, int64_t nchunks,
                                                                 void* __restrict__ out, const int* stop) {
  pack_EH_from_epart_body<PREC>(epart, nsplit, HC16, NB, K, G, scale, wgt, wmul, unscale_in, unscale_out, nchunks,
                                out, stop, blockIdx.x);
}

// The E^H-operand packing of E^H E in the lock-step batched solve (slice
// blockIdx.y of sl, as pack_data_E_batched_kernel).
template <int PREC>
__global__ __launch_bounds__(256) void pack_EH_from_epart_batched_kernel(const PackSlice* __restrict__ sl) {
  const PackSlice a = sl[blockIdx.y];
  if ((int64_t)blockIdx.x * 256 >= a.nchunks * a.NB * 64) return;
  pack_EH_from_epart_body<PREC>((const float*)a.src, a.nsplit, a.HC16, a.NB, a.n_items, a.G, a.scale, a.wgt, a.wmul,
                                a.unscale_in, a.unscale, a.nchunks, a.out, a.stop, blockIdx.x);
}

// ---------------------------------------------------------------------------
// The fused encode kernel.
//
// Grid: (ceil(HC / (kWaves * MT)), nsplit); 256 threads = 4 waves.  The
// linear workgroup id is remapped so that the workgroups the dispatcher
// places on one XCD (ids congruent mod 8) take a contiguous range of
// (split, held tile) pairs and so share their streamed chunks in that XCD's
// L2.  Wave w of workgroup x owns held tiles (x * 4 + w) * MT + [0, MT) and
// walks streamed chunks [split * cps, min(SC, (split + 1) * cps)); the 4
// waves share every streamed chunk through a double-buffered LDS stage
// filled by direct global-to-LDS loads one chunk ahead of its use.
//
// Per (held tile, streamed chunk):
//   1. phase tile on the f16 matrix cores: NQ x v_mfma_f32_16x16x32_f16
//      with A = streamed phase parts, B = held phase parts (see the packing
//      above).  Lane (g, j) ends up with phi for streamed items 4g + r
//      (r = 0..3) and held item j, in revolutions;
//   2. v_sin/v_cos (hardware, argument in revolutions), taken on the phase
//      directly while the bound sum_b max|a_b| max|h_b| (from the term
//      maxima, evaluated once per wave) stays below kRawPhaseBound, else
//      after v_fract; the hardware reduces an in-range argument itself, at
//      least as accurately as v_fract does;
//   3. these (cos, sin) pairs are exactly the A fragment of the complex
//      contraction (row = held item j, k-slots = streamed items 4g..4g+3 x
//      {cos, sin}), so they go to the matrix cores without any data movement:
//      one v_mfma_f32_16x16x32_{f16,bf16} per column block (two for bf16: hi
//      and lo data parts); FP32 splits the (cos, sin) operand as well and
//      takes the three products hi.lo, lo.hi, hi.hi of two-part f16
//      operands (three v_mfma_f32_16x16x32_f16 per column block, about
//      2^-21 relative per product, below the float32 phase's own error).
// Accumulators: lane (g, n) holds rows (held items) 4g + r, column 16 nb + n.
//
// Epilogue.  E: the partial y rows go to out_part[split][HC*16][NB*16].
// E^H: each lane forms conj(S) times its column's re or im part, the 16 lanes
// of a row group are summed with xor-shuffles (fixed order), and the
// coil-combined partial x goes to out_part (as float2) [split][HC*16].
// Operands of one streamed chunk as seen by one lane, read from LDS.
// The staged chunk is a sequence of 1 KB blocks, each [64 lanes][16 B]:
// NQ phase blocks, then the data blocks (NB blocks for fp16, 2 NB for bf16
// (hi, lo) and for fp32 (slots 0-3, 4-7)); lane l reads its 16 bytes of
// every block (conflict-free).
template <int PREC>
constexpr int data_blocks_per_nb() {
  return PREC == PREC_FP16 ? 1 : 2;
}

template <int PREC, int NB, int NQ>
struct Stream {
  static constexpr int NDB = NB * data_blocks_per_nb<PREC>();
  static constexpr int NBLK = NQ + NDB;
  u4 ph[NQ];
  u4 d[NDB];
  __device__ __forceinline__ void read(const u4* lds, int lane) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) ph[q] = lds[q * 64 + lane];
#pragma unroll
    for (int i = 0; i < NDB; ++i) d[i] = lds[(NQ + i) * 64 + lane];
  }
};

typedef __attribute__((address_space(3))) void lds_void;

// Wave `wave` copies blocks wave, wave + 4, ... of chunk ch into `dst`
// (global -> LDS directly, 16 bytes per lane, no registers involved).
template <int PREC, int NB, int NQ>
__device__ __forceinline__ void stage_chunk(const u4* __restrict__ strmcoef, const u4* __restrict__ sdata, int64_t ch,
                                            u4* dst, int wave, int lane) {
  constexpr int NDB = Stream<PREC, NB, NQ>::NDB;
  constexpr int NBLK = NQ + NDB;
#pragma unroll
  for (int blk = wave; blk < NBLK; blk += kWaves) {
    const u4* src = blk < NQ ? strmcoef + (ch * NQ + blk) * 64 + lane : sdata + (ch * NDB + (blk - NQ)) * 64 + lane;
    __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)(dst + blk * 64), 16, 0, 0);
  }
}

// The A operand of the contraction for one tile: the (cos, sin) pairs the
// lane holds, as FP16 (one part), BF16 (one part) or FP16 (two parts, for
// the FP32 form).
template <int PREC>
struct TileOperand {
  u4 hi, lo;  // lo used by the FP32 form only
};

// Phase tile on the f16 matrix cores: NQ chained 16x16x32 products.
template <int NQ>
__device__ __forceinline__ f4 phase_tile(const u4 (&ph)[NQ], const u4 (&hc)[NQ]) {
  f4 p = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < NQ; ++q)
    p = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, ph[q]), __builtin_bit_cast(h8, hc[q]), p, 0,
                                               0, 0);
  return p;
}

// sin/cos of a phase tile (revolutions; v_fract first when FRACT) and its
// conversion to the contraction operand.
template <int PREC, bool FRACT>
__device__ __forceinline__ TileOperand<PREC> tile_operand(f4 ph) {
  float cs[4], sn[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float x = FRACT ? __builtin_amdgcn_fractf(ph[r]) : ph[r];
    sn[r] = __builtin_amdgcn_sinf(x);
    cs[r] = __builtin_amdgcn_cosf(x);
  }
  TileOperand<PREC> op;
  if (PREC == PREC_FP16) {
    h8 a;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[2 * r] = (_Float16)cs[r];
      a[2 * r + 1] = (_Float16)sn[r];
    }
    op.hi = __builtin_bit_cast(u4, a);
    op.lo = u4{0, 0, 0, 0};
  } else if (PREC == PREC_BF16) {
    b8 a;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[2 * r] = (__bf16)cs[r];
      a[2 * r + 1] = (__bf16)sn[r];
    }
    op.hi = __builtin_bit_cast(u4, a);
    op.lo = u4{0, 0, 0, 0};
  } else {
    // (cos, sin) split: hi = both values rounded to f16 in one pack; lo =
    // x - hi, formed exactly by one mixed-precision FMA per value that reads
    // its half of the packed hi register, then rounded to f16
    h8 ahi, alo;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      typedef _Float16 h2 __attribute__((ext_vector_type(2)));
      h2 hp;
      hp[0] = (_Float16)cs[r];
      hp[1] = (_Float16)sn[r];
      const unsigned hb = __builtin_bit_cast(unsigned, hp);
      float lc, ls;
      asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(lc) : "v"(hb), "v"(cs[r]));
      asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(ls) : "v"(hb), "v"(sn[r]));
      ahi[2 * r] = hp[0];
      ahi[2 * r + 1] = hp[1];
      alo[2 * r] = (_Float16)lc;
      alo[2 * r + 1] = (_Float16)ls;
    }
    op.hi = __builtin_bit_cast(u4, ahi);
    op.lo = __builtin_bit_cast(u4, alo);
  }
  return op;
}

// The complex contraction of one tile against the streamed chunk's data
// operand: one 16x16x32 product per column block (FP16), two (BF16: hi and
// lo data parts), or three (FP32: lo.hi, hi.lo, hi.hi of two-part f16
// operands, summed from zero and added once on the VALU).
template <int PREC, int NB, int NQ>
__device__ __forceinline__ void contract_tile(const TileOperand<PREC>& op, const Stream<PREC, NB, NQ>& cur,
                                              f4 (&acc)[NB]) {
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    if (PREC == PREC_FP16) {
      acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, op.hi), __builtin_bit_cast(h8, cur.d[nb]),
                                                       acc[nb], 0, 0, 0);
    } else if (PREC == PREC_BF16) {
      acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, op.hi),
                                                        __builtin_bit_cast(b8, cur.d[2 * nb]), acc[nb], 0, 0, 0);
      acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, op.hi),
                                                        __builtin_bit_cast(b8, cur.d[2 * nb + 1]), acc[nb], 0, 0, 0);
    } else {
      const h8 dhi = __builtin_bit_cast(h8, cur.d[2 * nb]), dlo = __builtin_bit_cast(h8, cur.d[2 * nb + 1]);
      f4 t = {0.f, 0.f, 0.f, 0.f};
      t = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, op.lo), dhi, t, 0, 0, 0);
      t = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, op.hi), dlo, t, 0, 0, 0);
      t = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, op.hi), dhi, t, 0, 0, 0);
      acc[nb] += t;
    }
  }
}

// One (streamed chunk) x (MT held tiles) step: phase tiles, sin/cos, complex
// contraction into acc (see the kernel comment).
// FP16 and FP32 operands: software-pipelined across the held tiles: the
// phase products of all MT tiles are issued first, and the sin/cos of tile
// mt + 1 are formed before the contraction of tile mt, so that each tile's
// transcendentals can run on the VALU while the matrix cores work through
// the previous tile's contraction, and the phase results are long done by
// the time they are read (measured on the 3D and 2D workloads: 2-6 % less
// time per launch).  BF16 operands keep the tile-by-tile order, which
// measured faster for their two contraction products per column block.
// FRACT: reduce the phase with v_fract before the hardware sine/cosine
// (needed only when the phase may leave the +-256 revolution input range).
template <int PREC, int NB, int NQ, int MT, bool FRACT>
__device__ __forceinline__ void chunk_step(const Stream<PREC, NB, NQ>& cur, const u4 (&hc)[MT][NQ],
                                           f4 (&acc)[MT][NB]) {
  if (PREC == PREC_BF16) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      contract_tile<PREC, NB, NQ>(tile_operand<PREC, FRACT>(phase_tile<NQ>(cur.ph, hc[mt])), cur, acc[mt]);
    return;
  }
  f4 ph[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) ph[mt] = phase_tile<NQ>(cur.ph, hc[mt]);
  TileOperand<PREC> op = tile_operand<PREC, FRACT>(ph[0]);
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    TileOperand<PREC> next;
    if (mt + 1 < MT) next = tile_operand<PREC, FRACT>(ph[mt + 1]);
    contract_tile<PREC, NB, NQ>(op, cur, acc[mt]);
    if (mt + 1 < MT) op = next;
  }
}

// Epilogue of the contraction kernels.  E: the partial y rows go to
// out_part[split][HC*16][NB*16].  E^H: each lane forms conj(S) times its
// column's re or im part, the 16 lanes of a row group are summed with
// xor-shuffles (fixed order), and the coil-combined partial x goes to
// out_part (as float2) [split][HC*16].
template <int OP, int NB, int MT>
__device__ __forceinline__ void write_partials(const f4 (&acc)[MT][NB], int64_t tile0, int64_t split, int64_t HC,
                                               float* __restrict__ out_part, const float2* __restrict__ sens,
                                               int64_t L, int G, int lane) {
  const int g = lane >> 4, n = lane & 15;
  if (OP == OP_E) {
    float* o = out_part + (size_t)split * (size_t)HC * 16 * (NB * 16);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int64_t tile = tile0 + mt;
      if (tile >= HC) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = tile * 16 + g * 4 + r;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) o[row * (NB * 16) + nb * 16 + n] = acc[mt][nb][r];
      }
    }
  } else {
    float2* o = (float2*)out_part + (size_t)split * (size_t)HC * 16;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int64_t tile = tile0 + mt;
      if (tile >= HC) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t l = tile * 16 + g * 4 + r;
        float xr = 0.f, xi = 0.f;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const int N = nb * 16 + n;
          const int c = N >> 1;
          if (c < G && l < L) {
            const float2 s = sens[(int64_t)c * L + l];
            const float v = acc[mt][nb][r];
            if ((N & 1) == 0) {
              xr += s.x * v;
              xi -= s.y * v;
            } else {
              xr += s.y * v;
              xi += s.x * v;
            }
          }
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
          xr += __shfl_xor(xr, off);
          xi += __shfl_xor(xi, off);
        }
        if (n == r) o[l] = make_float2(xr, xi);
      }
    }
  }
}

// Walk streamed chunks [c0, c1) through the double-buffered LDS stage: the
// loads for chunk ch + 1 are issued right after the barrier that publishes
// chunk ch and overlap its compute.
template <int PREC, int NQ, int NB, int MT, bool FRACT>
__device__ __forceinline__ void stream_range(const u4* __restrict__ strmcoef, const u4* __restrict__ sd, int64_t c0,
                                             int64_t c1, const u4 (&hc)[MT][NQ], f4 (&acc)[MT][NB], u4* stage0,
                                             u4* stage1, int wave, int lane) {
  if (c0 < c1) stage_chunk<PREC, NB, NQ>(strmcoef, sd, c0, stage0, wave, lane);
  int buf = 0;
  for (int64_t ch = c0; ch < c1; ++ch) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of chunk ch have landed
    __syncthreads();                 // ... and every wave's; the other buffer is free
    if (ch + 1 < c1) stage_chunk<PREC, NB, NQ>(strmcoef, sd, ch + 1, buf ? stage0 : stage1, wave, lane);
    Stream<PREC, NB, NQ> cur;
    cur.read(buf ? stage1 : stage0, lane);
    chunk_step<PREC, NB, NQ, MT, FRACT>(cur, hc, acc);
    buf ^= 1;
  }
}

// One workgroup's share of an encode launch: held tiles
// (bx * kWaves + wave) * MT ... of one problem, over split `split` of the
// streamed chunks; st0, st1: the two LDS staging buffers.
template <int OP, int PREC, int NQ, int NB, int MT>
__device__ __forceinline__ void encode_block(const u4* __restrict__ heldcoef, const u4* __restrict__ strmcoef,
                                             const void* __restrict__ sdata, int64_t HC, int64_t SC, int64_t cps,
                                             float* __restrict__ out_part, const float2* __restrict__ sens,
                                             int64_t L, int G, const unsigned* __restrict__ tmax, int T, int64_t bx,
                                             int64_t split, u4* st0, u4* st1) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t tile0 = (bx * kWaves + wave) * MT;

  // bound on |phi| in revolutions: sum over terms of max|a_b| max|h_b|
  float bound = 0.f;
  if (lane < T) bound = __uint_as_float(tmax[lane]) * (float)kInv2Pi * __uint_as_float(tmax[kMaxTerms + lane]);
  for (int off = 32; off > 0; off >>= 1) bound += __shfl_xor(bound, off);
  const bool raw = bound < kRawPhaseBound;  // also false for NaN

  u4 hc[MT][NQ];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int64_t tile = tile0 + mt;
#pragma unroll
    for (int q = 0; q < NQ; ++q) hc[mt][q] = tile < HC ? heldcoef[(tile * NQ + q) * 64 + lane] : u4{0, 0, 0, 0};
  }
  // Accumulation: the matrix cores add straight into acc for the half
  // precisions (their operand rounding dominates); for FP32 the 3 MFMAs of a
  // chunk start from zero and their sum is added on the VALU, so the long
  // running sum is rounded once per chunk instead of once per MFMA.
  f4 acc[MT][NB];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mt][nb] = f4{0.f, 0.f, 0.f, 0.f};

  // Streamed chunks are staged through LDS, double-buffered and shared by
  // the 4 waves.
  const int64_t c0 = split * cps;
  const int64_t c1 = (c0 + cps < SC) ? c0 + cps : SC;
  const u4* sd = (const u4*)sdata;
  if (raw)
    stream_range<PREC, NQ, NB, MT, false>(strmcoef, sd, c0, c1, hc, acc, st0, st1, wave, lane);
  else
    stream_range<PREC, NQ, NB, MT, true>(strmcoef, sd, c0, c1, hc, acc, st0, st1, wave, lane);

  write_partials<OP, NB, MT>(acc, tile0, split, HC, out_part, sens, L, G, lane);
}

// XCD-aware order: block b of nblk goes to XCD b % 8 (round-robin dispatch);
// renumbering makes each XCD take a contiguous range of blocks, which share
// streamed chunks in that XCD's L2.
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t nblk) {
  const int64_t per = nblk / 8;
  return b < per * 8 ? (b % 8) * per + b / 8 : b;
}

template <int OP, int PREC, int NQ, int NB, int MT>
__global__ __launch_bounds__(256) void encode_kernel(
    const u4* __restrict__ heldcoef, const u4* __restrict__ strmcoef, const void* __restrict__ sdata, int64_t HC,
    int64_t SC, int64_t cps, float* __restrict__ out_part, const float2* __restrict__ sens, int64_t L, int G,
    const unsigned* __restrict__ tmax, int T, const int* stop) {
  if (stop && *stop) return;
  const int64_t b = xcd_order(blockIdx.x + (int64_t)gridDim.x * blockIdx.y, (int64_t)gridDim.x * gridDim.y);
  __shared__ u4 stage[2][Stream<PREC, NB, NQ>::NBLK * 64];
  encode_block<OP, PREC, NQ, NB, MT>(heldcoef, strmcoef, sdata, HC, SC, cps, out_part, sens, L, G, tmax, T,
                                     b % gridDim.x, b / gridDim.x, stage[0], stage[1]);
}

// Persistent form for many problems (slices) at once: a fixed grid takes the
// items of every slice's (held-tile block, split) work list in list order
// from an atomic counter (the host puts the longest items first), so one
// launch covers slices of different sizes (one launch per column-block
// count NB, which fixes the kernel's registers) and balances their uneven
// costs.  The loop ends for every workgroup once the counter passes the
// list's end.  Items of a slice whose stop flag is set are skipped.  Every
// item runs exactly the code of the single-problem kernel, so results are
// bit-identical to it.
template <int OP, int PREC, int NQ, int NB, int MT>
__global__ __launch_bounds__(256) void encode_persistent_kernel(EncodeBatch batch) {
  __shared__ u4 stage[2][Stream<PREC, NB, NQ>::NBLK * 64];
  __shared__ int next;
  const int64_t total = batch.total;
  for (;;) {
    __syncthreads();  // the previous item's reads of the staging buffers and of `next` are done
    if (threadIdx.x == 0) next = atomicAdd(batch.counter, 1);
    __syncthreads();
    const int64_t b = next;
    if (b >= total) break;
    int i = 0;
    while (i + 1 < batch.n && b >= batch.it[i + 1].first) ++i;
    const EncodeItem& e = batch.it[i];
    if (e.stop && *e.stop) continue;
    const int64_t lb = b - e.first;
    encode_block<OP, PREC, NQ, NB, MT>((const u4*)e.heldcoef, (const u4*)e.strmcoef, e.sdata, e.HC, e.SC, e.cps,
                                       e.out_part, e.sens, e.L, e.G, e.tmax, e.T, lb % e.gx, lb / e.gx, stage[0],
                                       stage[1]);
  }
}

// ---------------------------------------------------------------------------
// Resident P (the non-split form of the reconstruction figure): the (cos,
// sin) fragments of every (held tile, streamed chunk) pair are built once
// and kept in HBM, and every later E or E^H streams them instead of
// rebuilding them.  Layout, one array per direction:
//   P[(held tile * SC + streamed chunk) * 64 + lane] = 8 f16,
// the A fragment of the FP16 contraction exactly as the encode kernel forms
// it in registers (row = held item, k-slots = 4 streamed items x {cos, sin}).

// grid-stride over pairs, one wave per pair
template <int NQ>
__global__ __launch_bounds__(256) void build_P_kernel(const u4* __restrict__ heldcoef, const u4* __restrict__ strmcoef,
                                                      int64_t HC, int64_t SC, const unsigned* __restrict__ tmax,
                                                      int T, h8* __restrict__ P) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float bound = 0.f;
  if (lane < T) bound = __uint_as_float(tmax[lane]) * (float)kInv2Pi * __uint_as_float(tmax[kMaxTerms + lane]);
  for (int off = 32; off > 0; off >>= 1) bound += __shfl_xor(bound, off);
  const bool raw = bound < kRawPhaseBound;
  const int64_t npair = HC * SC;
  for (int64_t pair = (int64_t)blockIdx.x * kWaves + wave; pair < npair; pair += (int64_t)gridDim.x * kWaves) {
    const int64_t ht = pair / SC, ch = pair - ht * SC;
    f4 ph = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      ph = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, strmcoef[(ch * NQ + q) * 64 + lane]),
                                                  __builtin_bit_cast(h8, heldcoef[(ht * NQ + q) * 64 + lane]), ph, 0,
                                                  0, 0);
    h8 a;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float x = raw ? ph[r] : __builtin_amdgcn_fractf(ph[r]);
      a[2 * r] = (_Float16)__builtin_amdgcn_cosf(x);
      a[2 * r + 1] = (_Float16)__builtin_amdgcn_sinf(x);
    }
    P[pair * 64 + lane] = a;
  }
}

// The FP16 contraction against a resident P: same grid, split, LDS staging of
// the streamed data operand and epilogue as the encode kernel; the A
// fragments of the next chunk are loaded from P one chunk ahead.
template <int OP, int NB, int MT>
__global__ __launch_bounds__(256) void resident_kernel(const u4* __restrict__ P, const u4* __restrict__ sdata,
                                                       int64_t HC, int64_t SC, int64_t cps,
                                                       float* __restrict__ out_part, const float2* __restrict__ sens,
                                                       int64_t L, int G, const int* stop) {
  if (stop && *stop) return;
  const int64_t nblk = (int64_t)gridDim.x * gridDim.y;
  int64_t b = blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
  const int64_t per = nblk / 8;
  if (b < per * 8) b = (b % 8) * per + b / 8;
  const int64_t bx = b % gridDim.x;
  const int64_t split = b / gridDim.x;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t tile0 = (bx * kWaves + wave) * MT;

  f4 acc[MT][NB];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mt][nb] = f4{0.f, 0.f, 0.f, 0.f};
  __shared__ u4 stage[2][NB * 64];
  const int64_t c0 = split * cps;
  const int64_t c1 = (c0 + cps < SC) ? c0 + cps : SC;
  auto stage_data = [&](int64_t ch, u4* dst) {
#pragma unroll
    for (int blk = wave; blk < NB; blk += kWaves)
      __builtin_amdgcn_global_load_lds((const void*)(sdata + (ch * NB + blk) * 64 + lane), (lds_void*)(dst + blk * 64),
                                       16, 0, 0);
  };
  auto load_p = [&](int64_t ch, u4 (&pa)[MT]) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int64_t tile = tile0 + mt;
      pa[mt] = tile < HC ? P[(tile * SC + ch) * 64 + lane] : u4{0, 0, 0, 0};
    }
  };
  u4 pc[MT], pn[MT];
  if (c0 < c1) {
    stage_data(c0, stage[0]);
    load_p(c0, pc);
  }
  int buf = 0;
  for (int64_t ch = c0; ch < c1; ++ch) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of chunk ch (LDS copies and P) have landed
    __syncthreads();                 // ... and every wave's; the other buffer is free
    if (ch + 1 < c1) {
      stage_data(ch + 1, stage[buf ^ 1]);
      load_p(ch + 1, pn);
    }
    u4 d[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) d[nb] = stage[buf][nb * 64 + lane];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        acc[mt][nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, pc[mt]),
                                                             __builtin_bit_cast(h8, d[nb]), acc[mt][nb], 0, 0, 0);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) pc[mt] = pn[mt];
    buf ^= 1;
  }
  write_partials<OP, NB, MT>(acc, tile0, split, HC, out_part, sens, L, G, lane);
}

// ---------------------------------------------------------------------------
__global__ void finish_E_to_m_kernel(const float* __restrict__ epart, int nsplit, int64_t HC16, int NB,
                                     int64_t K, int G, const float* __restrict__ unscale,
                                     float2* __restrict__ m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K * G) return;
  const int64_t k = i % K;
  const int64_t c = i / K;
  const int ncol = NB * 16;
  const float2 v = sum_strided((const float2*)(epart + k * ncol + 2 * c), nsplit, HC16 * ncol / 2);
  const float u = unscale ? *unscale : 1.f;
  m[i] = make_float2(v.x * u, v.y * u);
}

__global__ void finish_EH_kernel(const float2* __restrict__ hpart, int nsplit, int64_t HC16, int64_t L,
                                 const float* __restrict__ unscale, float2* __restrict__ x) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  const float2 v = sum_strided(hpart + l, nsplit, HC16);
  const float u = unscale ? *unscale : 1.f;
  x[l] = make_float2(v.x * u, v.y * u);
}

// grad_b0[l] = Im(conj(rho[l]) x[l]), x = E^H (t o G) as split partials
__global__ void grad_b0_kernel(const float2* __restrict__ hpart, int nsplit, int64_t HC16, int64_t L,
                               const float* __restrict__ unscale, const float2* __restrict__ rho,
                               float* __restrict__ out) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  const float2 v = sum_strided(hpart + l, nsplit, HC16);
  const float u = unscale ? *unscale : 1.f;
  const float2 r = rho[l];
  out[l] = (r.x * v.y - r.y * v.x) * u;
}

// grad_kcoef[k][b] = Im(sum_c G[c][k] conj(Z[k][c])), Z = E (h_b o rho) as E partials
__global__ void grad_kcoef_kernel(const float* __restrict__ epart, int nsplit, int64_t HC16, int NB,
                                  const float* __restrict__ unscale, const float2* __restrict__ grad_m, int64_t K,
                                  int G, int P, int b, float* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int ncol = NB * 16;
  float acc = 0.f;
  for (int c = 0; c < G; ++c) {
    const float2 z = sum_strided((const float2*)(epart + k * ncol + 2 * c), nsplit, HC16 * ncol / 2);
    const float2 g = grad_m[(int64_t)c * K + k];
    acc += g.y * z.x - g.x * z.y;
  }
  out[k * P + b] = acc * (unscale ? *unscale : 1.f);
}

__global__ void fill_zero_kernel(float* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

__global__ void fill_kernel(float* __restrict__ p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// launchers
static inline dim3 grid1(int64_t n, int bs = 256) { return dim3((unsigned)cdiv(n, bs)); }

hipError_t launch_term_absmax(const float* t, const float* kcoef, int64_t K, const float* b0, const float* fields,
                              int64_t L, int P, unsigned* tmax, hipStream_t s) {
  hipError_t e = launch_fill_zero((float*)tmax, 2 * kMaxTerms, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(term_absmax_kernel, dim3(kTmaxBlocks, 2), dim3(256), 0, s, t, kcoef, K, b0, fields, L, P, tmax);
  return hipGetLastError();
}

hipError_t launch_pack_phase(const float* c0, const float* cb, int64_t n_items, int P, int side, int role, int NQ,
                             const unsigned* tmax, void* out, hipStream_t s) {
  const int64_t total = cdiv(n_items, kChunk) * NQ * 64;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(pack_phase_kernel, grid1(total), dim3(256), 0, s, c0, cb, n_items, P, side, role, NQ, tmax,
                     (h8*)out, total);
  return hipGetLastError();
}

hipError_t launch_scale_sens(const float2* sens, const float* icorr, int G, int64_t L, float2* out,
                             hipStream_t s) {
  if ((int64_t)G * L == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_sens_kernel, grid1((int64_t)G * L), dim3(256), 0, s, sens, icorr, G, L, out);
  return hipGetLastError();
}

hipError_t launch_absmax(const float2* src, const float2* mul, const float* wgt, int64_t n_items, int64_t is,
                         int64_t cs, int G, float* bmax, const int* stop, hipStream_t s) {
  hipLaunchKernelGGL(absmax_kernel, dim3(kBmaxBlocks), dim3(256), 0, s, src, mul, wgt, n_items, is, cs, G, bmax,
                     stop);
  return hipGetLastError();
}

hipError_t launch_pack_data(int op, int prec, const float2* src, const float2* mul, const float* wgt, int64_t n_items,
                            int64_t is, int64_t cs, int G, int NB, int64_t nchunks, void* out, const float* bmax,
                            float* unscale, const int* stop, hipStream_t s) {
  const int64_t total = nchunks * NB * 64;
  if (total == 0) return hipSuccess;
  const dim3 gr = grid1(total), bl(256);
#define NFS_PACK(P_, O_)                                                                                   \
  hipLaunchKernelGGL((pack_data_kernel<P_, O_>), gr, bl, 0, s, src, mul, wgt, n_items, is, cs, G, NB, nchunks, \
                     out, bmax, unscale, stop)
  if (op == OP_E) {
    if (prec == PREC_FP32) NFS_PACK(PREC_FP32, OP_E);
    else if (prec == PREC_BF16) NFS_PACK(PREC_BF16, OP_E);
    else NFS_PACK(PREC_FP16, OP_E);
  } else {
    if (prec == PREC_FP32) NFS_PACK(PREC_FP32, OP_EH);
    else if (prec == PREC_BF16) NFS_PACK(PREC_BF16, OP_EH);
    else NFS_PACK(PREC_FP16, OP_EH);
  }
#undef NFS_PACK
  return hipGetLastError();
}

template <int OP, int PREC, int NQ, int NB, int MT>
static hipError_t launch_encode_t(const EncodeShape& sh, const void* heldcoef, const void* strmcoef,
                                  const void* sdata, float* out_part, const float2* sens, int64_t L, int G,
                                  const unsigned* tmax, int T, const int* stop, hipStream_t s) {
  const dim3 gr((unsigned)cdiv(sh.HC, (int64_t)kWaves * MT), (unsigned)sh.nsplit);
  hipLaunchKernelGGL((encode_kernel<OP, PREC, NQ, NB, MT>), gr, dim3(64 * kWaves), 0, s, (const u4*)heldcoef,
                     (const u4*)strmcoef, sdata, sh.HC, sh.SC, sh.cps, out_part, sens, L, G, tmax, T, stop);
  return hipGetLastError();
}

#define NFS_ENC_ARGS sh, hc, scf, sd, op, sens, L, G, tmax, T, stop, s
template <int OP, int PREC, int NQ>
static hipError_t launch_encode_nb(const EncodeShape& sh, const void* hc, const void* scf, const void* sd, float* op,
                                   const float2* sens, int64_t L, int G, const unsigned* tmax, int T, const int* stop,
                                   hipStream_t s) {
  const int k = sh.NB * 8 + sh.MT;
  switch (k) {
    case 1 * 8 + 2: return launch_encode_t<OP, PREC, NQ, 1, 2>(NFS_ENC_ARGS);
    case 1 * 8 + 4: return launch_encode_t<OP, PREC, NQ, 1, 4>(NFS_ENC_ARGS);
    case 2 * 8 + 2: return launch_encode_t<OP, PREC, NQ, 2, 2>(NFS_ENC_ARGS);
    case 2 * 8 + 4: return launch_encode_t<OP, PREC, NQ, 2, 4>(NFS_ENC_ARGS);
    case 4 * 8 + 2: return launch_encode_t<OP, PREC, NQ, 4, 2>(NFS_ENC_ARGS);
    case 4 * 8 + 4: return launch_encode_t<OP, PREC, NQ, 4, 4>(NFS_ENC_ARGS);
    case 8 * 8 + 2: return launch_encode_t<OP, PREC, NQ, 8, 2>(NFS_ENC_ARGS);
  }
  return hipErrorInvalidValue;
}

template <int OP, int PREC>
static hipError_t launch_encode_nq(const EncodeShape& sh, const void* hc, const void* scf, const void* sd, float* op,
                                   const float2* sens, int64_t L, int G, const unsigned* tmax, int T, const int* stop,
                                   hipStream_t s) {
  switch (sh.NQ) {
    case 1: return launch_encode_nb<OP, PREC, 1>(NFS_ENC_ARGS);
    case 2: return launch_encode_nb<OP, PREC, 2>(NFS_ENC_ARGS);
    case 3: return launch_encode_nb<OP, PREC, 3>(NFS_ENC_ARGS);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_encode(const EncodeShape& sh, const void* hc, const void* scf, const void* sd, float* op,
                         const float2* sens, int64_t L, int G, const unsigned* tmax, int T, const int* stop,
                         hipStream_t s) {
  if (sh.HC == 0) return hipSuccess;
  if (!valid_held_tiles(sh.NB, sh.MT) || sh.nsplit < 1 || T < 1 || T > kMaxTerms) return hipErrorInvalidValue;
  if (sh.op == OP_E) {
    if (sh.prec == PREC_FP32) return launch_encode_nq<OP_E, PREC_FP32>(NFS_ENC_ARGS);
    if (sh.prec == PREC_BF16) return launch_encode_nq<OP_E, PREC_BF16>(NFS_ENC_ARGS);
    return launch_encode_nq<OP_E, PREC_FP16>(NFS_ENC_ARGS);
  }
  if (sh.prec == PREC_FP32) return launch_encode_nq<OP_EH, PREC_FP32>(NFS_ENC_ARGS);
  if (sh.prec == PREC_BF16) return launch_encode_nq<OP_EH, PREC_BF16>(NFS_ENC_ARGS);
  return launch_encode_nq<OP_EH, PREC_FP16>(NFS_ENC_ARGS);
}
#undef NFS_ENC_ARGS

template <int OP, int PREC, int NQ>
static hipError_t launch_persistent_nb(const EncodeBatch& b, int NB, int MT, int grid, hipStream_t s) {
  switch (NB * 8 + MT) {
#define NFS_PERSIST(nb, mt)                                                                                       \
  case nb * 8 + mt:                                                                                             \
    hipLaunchKernelGGL((encode_persistent_kernel<OP, PREC, NQ, nb, mt>), dim3(grid), dim3(256), 0, s, b); \
    break;
    NFS_PERSIST(1, 2)
    NFS_PERSIST(1, 4)
    NFS_PERSIST(2, 2)
    NFS_PERSIST(2, 4)
    NFS_PERSIST(4, 2)
    NFS_PERSIST(4, 4)
#undef NFS_PERSIST
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int OP, int PREC>
static hipError_t launch_persistent_nq(const EncodeBatch& b, int NQ, int NB, int MT, int grid, hipStream_t s) {
  if (NQ == 1) return launch_persistent_nb<OP, PREC, 1>(b, NB, MT, grid, s);
  if (NQ == 2) return launch_persistent_nb<OP, PREC, 2>(b, NB, MT, grid, s);
  return hipErrorInvalidValue;
}

bool persistent_supported(int prec, int NQ, int NB, int MT) {
  return (prec == PREC_FP16 || prec == PREC_BF16) && (NQ == 1 || NQ == 2) && (NB == 1 || NB == 2 || NB == 4) &&
         valid_held_tiles(NB, MT);
}

hipError_t launch_encode_persistent(int op, int prec, int NQ, int NB, int MT, const EncodeBatch& b, int grid,
                                    hipStream_t s) {
  if (b.total == 0) return hipSuccess;
  if (b.n < 1 || b.n > kMaxBatchItems || grid < 1 || !b.counter || !persistent_supported(prec, NQ, NB, MT) ||
      b.total > INT32_MAX)
    return hipErrorInvalidValue;
  for (int i = 0; i < b.n; ++i)
    if (b.it[i].NB != NB || b.it[i].T < 1 || b.it[i].T > kMaxTerms) return hipErrorInvalidValue;
  if (op == OP_E)
    return prec == PREC_BF16 ? launch_persistent_nq<OP_E, PREC_BF16>(b, NQ, NB, MT, grid, s)
                             : launch_persistent_nq<OP_E, PREC_FP16>(b, NQ, NB, MT, grid, s);
  return prec == PREC_BF16 ? launch_persistent_nq<OP_EH, PREC_BF16>(b, NQ, NB, MT, grid, s)
                           : launch_persistent_nq<OP_EH, PREC_FP16>(b, NQ, NB, MT, grid, s);
}

hipError_t launch_build_P(int NQ, const void* heldcoef, const void* strmcoef, int64_t HC, int64_t SC,
                          const unsigned* tmax, int T, void* P, hipStream_t s) {
  const int64_t npair = HC * SC;
  if (npair == 0) return hipSuccess;
  const dim3 gr((unsigned)std::min<int64_t>(cdiv(npair, kWaves), 1 << 20)), bl(64 * kWaves);
  switch (NQ) {
    case 1: hipLaunchKernelGGL(build_P_kernel<1>, gr, bl, 0, s, (const u4*)heldcoef, (const u4*)strmcoef, HC, SC, tmax, T, (h8*)P); break;
    case 2: hipLaunchKernelGGL(build_P_kernel<2>, gr, bl, 0, s, (const u4*)heldcoef, (const u4*)strmcoef, HC, SC, tmax, T, (h8*)P); break;
    case 3: hipLaunchKernelGGL(build_P_kernel<3>, gr, bl, 0, s, (const u4*)heldcoef, (const u4*)strmcoef, HC, SC, tmax, T, (h8*)P); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int OP, int NB, int MT>
static hipError_t launch_resident_t(const EncodeShape& sh, const void* P, const void* sdata, float* out_part,
                                    const float2* sens, int64_t L, int G, const int* stop, hipStream_t s) {
  const dim3 gr((unsigned)cdiv(sh.HC, (int64_t)kWaves * MT), (unsigned)sh.nsplit);
  hipLaunchKernelGGL((resident_kernel<OP, NB, MT>), gr, dim3(64 * kWaves), 0, s, (const u4*)P, (const u4*)sdata,
                     sh.HC, sh.SC, sh.cps, out_part, sens, L, G, stop);
  return hipGetLastError();
}

template <int OP>
static hipError_t launch_resident_op(const EncodeShape& sh, const void* P, const void* sd, float* op,
                                     const float2* sens, int64_t L, int G, const int* stop, hipStream_t s) {
  switch (sh.NB * 8 + sh.MT) {
    case 1 * 8 + 2: return launch_resident_t<OP, 1, 2>(sh, P, sd, op, sens, L, G, stop, s);
    case 1 * 8 + 4: return launch_resident_t<OP, 1, 4>(sh, P, sd, op, sens, L, G, stop, s);
    case 2 * 8 + 2: return launch_resident_t<OP, 2, 2>(sh, P, sd, op, sens, L, G, stop, s);
    case 2 * 8 + 4: return launch_resident_t<OP, 2, 4>(sh, P, sd, op, sens, L, G, stop, s);
    case 4 * 8 + 2: return launch_resident_t<OP, 4, 2>(sh, P, sd, op, sens, L, G, stop, s);
    case 4 * 8 + 4: return launch_resident_t<OP, 4, 4>(sh, P, sd, op, sens, L, G, stop, s);
    case 8 * 8 + 2: return launch_resident_t<OP, 8, 2>(sh, P, sd, op, sens, L, G, stop, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_resident(const EncodeShape& sh, const void* P, const void* sdata, float* out_part,
                           const float2* sens, int64_t L, int G, const int* stop, hipStream_t s) {
  if (sh.HC == 0) return hipSuccess;
  if (sh.prec != PREC_FP16 || !valid_held_tiles(sh.NB, sh.MT) || sh.nsplit < 1) return hipErrorInvalidValue;
  return sh.op == OP_E ? launch_resident_op<OP_E>(sh, P, sdata, out_part, sens, L, G, stop, s)
                       : launch_resident_op<OP_EH>(sh, P, sdata, out_part, sens, L, G, stop, s);
}

hipError_t launch_finish_E_to_m(const float* epart, int nsplit, int64_t HC16, int NB, int64_t K, int G,
                                const float* unscale, float2* m, hipStream_t s) {
  if (K * G == 0) return hipSuccess;
  hipLaunchKernelGGL(finish_E_to_m_kernel, grid1(K * G), dim3(256), 0, s, epart, nsplit, HC16, NB, K, G, unscale, m);
  return hipGetLastError();
}

float epart_pack_scale(int prec, int64_t L) {
  int lg = 0;
  while (((int64_t)1 << lg) < L) ++lg;
  return prec != PREC_BF16 ? ldexpf(1.f, -(lg + 1)) : 1.f;
}

hipError_t launch_pack_EH_from_epart(int prec, const float* epart, int nsplit, int64_t HC16, int NB, int64_t K, int G,
                                     int64_t L, const float* wgt, float wmul, const float* unscale_in,
                                     float* unscale_out, int64_t nchunks, void* out, const int* stop, hipStream_t s) {
  const int64_t total = nchunks * NB * 64;
  if (total == 0) return hipSuccess;
  const float scale = epart_pack_scale(prec, L);
  const dim3 gr = grid1(total), bl(256);
#define NFS_PACKH(P_)                                                                                           \
  hipLaunchKernelGGL(pack_EH_from_epart_kernel<P_>, gr, bl, 0, s, epart, nsplit, HC16, NB, K, G, scale, wgt, wmul, \
                     unscale_in, unscale_out, nchunks, out, stop)
  if (prec == PREC_FP32) NFS_PACKH(PREC_FP32);
  else if (prec == PREC_BF16) NFS_PACKH(PREC_BF16);
  else NFS_PACKH(PREC_FP16);
#undef NFS_PACKH
  return hipGetLastError();
}

hipError_t launch_pack_EH_from_epart_batched(int prec, const PackSlice* sl, int n, int64_t max_blocks,
                                             hipStream_t s) {
  if (n == 0 || max_blocks == 0) return hipSuccess;
  const dim3 gr((unsigned)max_blocks, (unsigned)n), bl(256);
  if (prec == PREC_FP32) hipLaunchKernelGGL(pack_EH_from_epart_batched_kernel<PREC_FP32>, gr, bl, 0, s, sl);
  else if (prec == PREC_BF16) hipLaunchKernelGGL(pack_EH_from_epart_batched_kernel<PREC_BF16>, gr, bl, 0, s, sl);
  else hipLaunchKernelGGL(pack_EH_from_epart_batched_kernel<PREC_FP16>, gr, bl, 0, s, sl);
  return hipGetLastError();
}

hipError_t launch_pack_data_E_batched(int prec, const PackSlice* sl, int n, int64_t max_blocks, hipStream_t s) {
  if (n == 0 || max_blocks == 0) return hipSuccess;
  const dim3 gr((unsigned)max_blocks, (unsigned)n), bl(256);
  if (prec == PREC_FP32) hipLaunchKernelGGL(pack_data_E_batched_kernel<PREC_FP32>, gr, bl, 0, s, sl);
  else if (prec == PREC_BF16) hipLaunchKernelGGL(pack_data_E_batched_kernel<PREC_BF16>, gr, bl, 0, s, sl);
  else hipLaunchKernelGGL(pack_data_E_batched_kernel<PREC_FP16>, gr, bl, 0, s, sl);
  return hipGetLastError();
}

hipError_t launch_finish_EH(const float2* hpart, int nsplit, int64_t HC16, int64_t L, const float* unscale,
                            float2* x, hipStream_t s) {
  if (L == 0) return hipSuccess;
  hipLaunchKernelGGL(finish_EH_kernel, grid1(L), dim3(256), 0, s, hpart, nsplit, HC16, L, unscale, x);
  return hipGetLastError();
}

hipError_t launch_grad_b0(const float2* hpart, int nsplit, int64_t HC16, int64_t L, const float* unscale,
                          const float2* rho, float* out, hipStream_t s) {
  if (L == 0) return hipSuccess;
  hipLaunchKernelGGL(grad_b0_kernel, grid1(L), dim3(256), 0, s, hpart, nsplit, HC16, L, unscale, rho, out);
  return hipGetLastError();
}

hipError_t launch_grad_kcoef(const float* epart, int nsplit, int64_t HC16, int NB, const float* unscale,
                             const float2* grad_m, int64_t K, int G, int P, int b, float* out, hipStream_t s) {
  if (K == 0) return hipSuccess;
  hipLaunchKernelGGL(grad_kcoef_kernel, grid1(K), dim3(256), 0, s, epart, nsplit, HC16, NB, unscale, grad_m, K, G, P,
                     b, out);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, grid1(n), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, grid1(n), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace nfs
