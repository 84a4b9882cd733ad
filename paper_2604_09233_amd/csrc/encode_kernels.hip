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
#include "nfs_internal.h"

namespace nfs {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr double kInv2Pi = 0.159154943091895335768883763372514362;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---------------------------------------------------------------------------
// Phase coefficients in MFMA fragment order.
// out[(chunk * NT + tg) * 64 + lane] = coef[item = 16 chunk + lane % 16][term = 4 tg + lane / 16]
// This is the per-lane operand of v_mfma_f32_16x16x4_f32 for both the A side
// (row = lane % 16, k = lane / 16) and the B side (k = lane / 16,
// column = lane % 16), so one packed array serves either role.
// Sample side: term 0 = t, term b+1 = kcoef[.][b], both scaled to revolutions.
// Voxel side:  term 0 = b0, term b+1 = fields[b][.].
__global__ void pack_coef_samples_kernel(const float* __restrict__ kcoef, const float* __restrict__ t,
                                         int64_t K, int P, int NT, float* __restrict__ out,
                                         int64_t total) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int lane = (int)(i & 63);
  const int64_t q = i >> 6;
  const int tg = (int)(q % NT);
  const int64_t chunk = q / NT;
  const int64_t k = chunk * kChunk + (lane & 15);
  const int term = tg * 4 + (lane >> 4);
  float v = 0.f;
  if (k < K) {
    if (term == 0)
      v = (float)((double)t[k] * kInv2Pi);
    else if (term <= P)
      v = (float)((double)kcoef[k * P + (term - 1)] * kInv2Pi);
  }
  out[i] = v;
}

__global__ void pack_coef_voxels_kernel(const float* __restrict__ fields, const float* __restrict__ b0,
                                        int64_t L, int P, int NT, float* __restrict__ out,
                                        int64_t total) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int lane = (int)(i & 63);
  const int64_t q = i >> 6;
  const int tg = (int)(q % NT);
  const int64_t chunk = q / NT;
  const int64_t l = chunk * kChunk + (lane & 15);
  const int term = tg * 4 + (lane >> 4);
  float v = 0.f;
  if (l < L) {
    if (term == 0)
      v = b0[l];
    else if (term <= P)
      v = fields[(int64_t)(term - 1) * L + l];
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
// Largest |re| or |im| of value(item, c) = src[item*is + c*cs] * mul[c][item]
// per workgroup (kBmaxBlocks workgroups, every entry of bmax written).
__global__ __launch_bounds__(256) void absmax_kernel(const float2* __restrict__ src,
                                                     const float2* __restrict__ mul, int64_t n_items,
                                                     int64_t is, int64_t cs, int G,
                                                     float* __restrict__ bmax, const int* stop) {
  if (stop && *stop) return;
  __shared__ float red[256];
  float mx = 0.f;
  for (int64_t item = (int64_t)blockIdx.x * 256 + threadIdx.x; item < n_items;
       item += (int64_t)gridDim.x * 256) {
    for (int c = 0; c < G; ++c) {
      float2 v = src[item * is + (int64_t)c * cs];
      if (mul) v = cmul(mul[(int64_t)c * n_items + item], v);
      mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
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
//   fp32: [((ch*NB + nb)*8 + u)*64 + lane]
// FP16: the values are scaled by a power of two so that the largest
// magnitude lands just below 2^14; 1/scale is stored in *unscale.
template <int PREC, int OP>
__global__ __launch_bounds__(256) void pack_data_kernel(
    const float2* __restrict__ src, const float2* __restrict__ mul, int64_t n_items, int64_t is,
    int64_t cs, int G, int NB, int64_t nchunks, void* __restrict__ out, const float* __restrict__ bmax,
    float* __restrict__ unscale, const int* stop) {
  if (stop && *stop) return;
  float scale = 1.f;
  if (PREC == PREC_FP16) {
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
    if (blockIdx.x == 0 && threadIdx.x == 0) *unscale = 1.f / scale;
  }
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
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
      v.x *= scale;
      v.y *= scale;
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
  if (PREC == PREC_FP32) {
    float* o = (float*)out;
#pragma unroll
    for (int u = 0; u < 8; ++u) o[((ch * NB + nb) * 8 + u) * 64 + lane] = vals[u];
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
// The fused encode kernel.
//
// Grid: (ceil(HC / (kWaves * MT)), nsplit); 256 threads = 4 waves.  The
// linear workgroup id is remapped so that the workgroups the dispatcher
// places on one XCD (ids congruent mod 8) take a contiguous range of
// (split, held tile) pairs and so share their streamed chunks in that XCD's
// L2.  Wave w of workgroup x owns held tiles (x * 4 + w) * MT + [0, MT) and
// walks streamed chunks [split * cps, min(SC, (split + 1) * cps)).
//
// Per (held tile, streamed chunk):
//   1. phase tile on the FP32 matrix cores: NT x v_mfma_f32_16x16x4_f32 with
//      A = streamed coefficients, B = held coefficients.  Lane (g, j) ends up
//      with phi for streamed items 4g + r (r = 0..3) and held item j, in
//      revolutions;
//   2. v_fract + v_sin/v_cos (hardware, argument in revolutions);
//   3. these (cos, sin) pairs are exactly the A fragment of the complex
//      contraction (row = held item j, k-slots = streamed items 4g..4g+3 x
//      {cos, sin}), so they go to the matrix cores without any data movement:
//      one v_mfma_f32_16x16x32_{f16,bf16} per column block, or 8
//      v_mfma_f32_16x16x4_f32 per column block for FP32.
// Accumulators: lane (g, n) holds rows (held items) 4g + r, column 16 nb + n.
//
// Epilogue.  E: the partial y rows go to out_part[split][HC*16][NB*16].
// E^H: each lane forms conj(S) times its column's re or im part, the 16 lanes
// of a row group are summed with xor-shuffles (fixed order), and the
// coil-combined partial x goes to out_part (as float2) [split][HC*16].
template <int OP, int PREC, int NT, int NB, int MT>
__global__ __launch_bounds__(256) void encode_kernel(
    const float* __restrict__ heldcoef, const float* __restrict__ strmcoef,
    const void* __restrict__ sdata, int64_t HC, int64_t SC, int64_t cps, float* __restrict__ out_part,
    const float2* __restrict__ sens, int64_t L, int G, const int* stop) {
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

  float hc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int64_t tile = tile0 + mt;
#pragma unroll
    for (int t = 0; t < NT; ++t) hc[mt][t] = tile < HC ? heldcoef[(tile * NT + t) * 64 + lane] : 0.f;
  }
  // Two-level accumulation: the matrix cores add into `inner`, which is
  // flushed into `acc` on the VALU every IC chunks, so the long running sum
  // is rounded once per IC chunks instead of once per MFMA.
  constexpr int IC = PREC == PREC_FP32 ? 1 : 8;
  f4 acc[MT][NB], inner[MT][NB];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      acc[mt][nb] = f4{0.f, 0.f, 0.f, 0.f};
      inner[mt][nb] = f4{0.f, 0.f, 0.f, 0.f};
    }
  int since_flush = 0;

  const int64_t c0 = split * cps;
  const int64_t c1 = (c0 + cps < SC) ? c0 + cps : SC;
  for (int64_t ch = c0; ch < c1; ++ch) {
    float sc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) sc[t] = strmcoef[(ch * NT + t) * 64 + lane];
    constexpr int NFRAG = PREC == PREC_BF16 ? 2 : 1;
    u4 bh[PREC == PREC_FP32 ? 1 : NB][NFRAG];
    float bf[PREC == PREC_FP32 ? NB : 1][8];
    if (PREC == PREC_FP32) {
      const float* d = (const float*)sdata;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int u = 0; u < 8; ++u) bf[nb][u] = d[((ch * NB + nb) * 8 + u) * 64 + lane];
    } else {
      const u4* d = (const u4*)sdata;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int f = 0; f < NFRAG; ++f) bh[nb][f] = d[((ch * NB + nb) * NFRAG + f) * 64 + lane];
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      f4 ph = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < NT; ++t) ph = __builtin_amdgcn_mfma_f32_16x16x4f32(sc[t], hc[mt][t], ph, 0, 0, 0);
      float cs[4], sn[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float x = __builtin_amdgcn_fractf(ph[r]);
        sn[r] = __builtin_amdgcn_sinf(x);
        cs[r] = __builtin_amdgcn_cosf(x);
      }
      if (PREC == PREC_FP16) {
        h8 a;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          a[2 * r] = (_Float16)cs[r];
          a[2 * r + 1] = (_Float16)sn[r];
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          inner[mt][nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, __builtin_bit_cast(h8, bh[nb][0]), inner[mt][nb], 0, 0, 0);
      } else if (PREC == PREC_BF16) {
        b8 a;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          a[2 * r] = (__bf16)cs[r];
          a[2 * r + 1] = (__bf16)sn[r];
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          inner[mt][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(b8, bh[nb][0]), inner[mt][nb], 0, 0, 0);
          inner[mt][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(b8, bh[nb][NFRAG - 1]), inner[mt][nb], 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const float a = (u & 1) ? sn[u >> 1] : cs[u >> 1];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            inner[mt][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bf[nb][u], inner[mt][nb], 0, 0, 0);
        }
      }
    }
    if (++since_flush == IC) {
      since_flush = 0;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          acc[mt][nb] += inner[mt][nb];
          inner[mt][nb] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[mt][nb] += inner[mt][nb];

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

// ---------------------------------------------------------------------------
__global__ void finish_E_to_m_kernel(const float* __restrict__ epart, int nsplit, int64_t HC16, int NB,
                                     int64_t K, int G, const float* __restrict__ unscale,
                                     float2* __restrict__ m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K * G) return;
  const int64_t k = i % K;
  const int64_t c = i / K;
  const int ncol = NB * 16;
  float re = 0.f, im = 0.f;
  for (int s = 0; s < nsplit; ++s) {
    const float* row = epart + ((size_t)s * HC16 + k) * ncol;
    re += row[2 * c];
    im += row[2 * c + 1];
  }
  const float u = unscale ? *unscale : 1.f;
  m[i] = make_float2(re * u, im * u);
}

__global__ void finish_E_to_ybuf_kernel(const float* __restrict__ epart, int nsplit, int64_t n,
                                        const float* __restrict__ unscale, float* __restrict__ ybuf,
                                        const int* stop) {
  if (stop && *stop) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float v = 0.f;
  for (int s = 0; s < nsplit; ++s) v += epart[(size_t)s * n + i];
  ybuf[i] = v * (unscale ? *unscale : 1.f);
}

__global__ void finish_EH_kernel(const float2* __restrict__ hpart, int nsplit, int64_t HC16, int64_t L,
                                 const float* __restrict__ unscale, float2* __restrict__ x) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= L) return;
  float re = 0.f, im = 0.f;
  for (int s = 0; s < nsplit; ++s) {
    const float2 v = hpart[(size_t)s * HC16 + l];
    re += v.x;
    im += v.y;
  }
  const float u = unscale ? *unscale : 1.f;
  x[l] = make_float2(re * u, im * u);
}

__global__ void fill_zero_kernel(float* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// ---------------------------------------------------------------------------
// launchers
static inline dim3 grid1(int64_t n, int bs = 256) { return dim3((unsigned)cdiv(n, bs)); }

hipError_t launch_pack_coef_samples(const float* kcoef, const float* t, int64_t K, int P, int NT, float* out,
                                    hipStream_t s) {
  const int64_t total = cdiv(K, kChunk) * NT * 64;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(pack_coef_samples_kernel, grid1(total), dim3(256), 0, s, kcoef, t, K, P, NT, out, total);
  return hipGetLastError();
}

hipError_t launch_pack_coef_voxels(const float* fields, const float* b0, int64_t L, int P, int NT, float* out,
                                   hipStream_t s) {
  const int64_t total = cdiv(L, kChunk) * NT * 64;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(pack_coef_voxels_kernel, grid1(total), dim3(256), 0, s, fields, b0, L, P, NT, out, total);
  return hipGetLastError();
}

hipError_t launch_scale_sens(const float2* sens, const float* icorr, int G, int64_t L, float2* out,
                             hipStream_t s) {
  if ((int64_t)G * L == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_sens_kernel, grid1((int64_t)G * L), dim3(256), 0, s, sens, icorr, G, L, out);
  return hipGetLastError();
}

hipError_t launch_absmax(const float2* src, const float2* mul, int64_t n_items, int64_t is, int64_t cs, int G,
                         float* bmax, const int* stop, hipStream_t s) {
  hipLaunchKernelGGL(absmax_kernel, dim3(kBmaxBlocks), dim3(256), 0, s, src, mul, n_items, is, cs, G, bmax, stop);
  return hipGetLastError();
}

hipError_t launch_pack_data(int op, int prec, const float2* src, const float2* mul, int64_t n_items, int64_t is,
                            int64_t cs, int G, int NB, int64_t nchunks, void* out, const float* bmax,
                            float* unscale, const int* stop, hipStream_t s) {
  const int64_t total = nchunks * NB * 64;
  if (total == 0) return hipSuccess;
  const dim3 gr = grid1(total), bl(256);
#define NFS_PACK(P_, O_)                                                                                   \
  hipLaunchKernelGGL((pack_data_kernel<P_, O_>), gr, bl, 0, s, src, mul, n_items, is, cs, G, NB, nchunks, \
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

template <int OP, int PREC, int NT, int NB, int MT>
static hipError_t launch_encode_t(const EncodeShape& sh, const float* heldcoef, const float* strmcoef,
                                  const void* sdata, float* out_part, const float2* sens, int64_t L, int G,
                                  const int* stop, hipStream_t s) {
  const dim3 gr((unsigned)cdiv(sh.HC, (int64_t)kWaves * MT), (unsigned)sh.nsplit);
  hipLaunchKernelGGL((encode_kernel<OP, PREC, NT, NB, MT>), gr, dim3(64 * kWaves), 0, s, heldcoef, strmcoef,
                     sdata, sh.HC, sh.SC, sh.cps, out_part, sens, L, G, stop);
  return hipGetLastError();
}

template <int OP, int PREC, int NT>
static hipError_t launch_encode_nb(const EncodeShape& sh, const float* hc, const float* scf, const void* sd,
                                   float* op, const float2* sens, int64_t L, int G, const int* stop,
                                   hipStream_t s) {
  switch (sh.NB) {
    case 1: return launch_encode_t<OP, PREC, NT, 1, 2>(sh, hc, scf, sd, op, sens, L, G, stop, s);
    case 2: return launch_encode_t<OP, PREC, NT, 2, 2>(sh, hc, scf, sd, op, sens, L, G, stop, s);
    case 4: return launch_encode_t<OP, PREC, NT, 4, 2>(sh, hc, scf, sd, op, sens, L, G, stop, s);
    case 8: return launch_encode_t<OP, PREC, NT, 8, 2>(sh, hc, scf, sd, op, sens, L, G, stop, s);
  }
  return hipErrorInvalidValue;
}

template <int OP, int PREC>
static hipError_t launch_encode_nt(const EncodeShape& sh, const float* hc, const float* scf, const void* sd,
                                   float* op, const float2* sens, int64_t L, int G, const int* stop,
                                   hipStream_t s) {
  switch (sh.NT) {
    case 2: return launch_encode_nb<OP, PREC, 2>(sh, hc, scf, sd, op, sens, L, G, stop, s);
    case 5: return launch_encode_nb<OP, PREC, 5>(sh, hc, scf, sd, op, sens, L, G, stop, s);
    case 8: return launch_encode_nb<OP, PREC, 8>(sh, hc, scf, sd, op, sens, L, G, stop, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_encode(const EncodeShape& sh, const float* heldcoef, const float* strmcoef, const void* sdata,
                         float* out_part, const float2* sens, int64_t L, int G, const int* stop, hipStream_t s) {
  if (sh.HC == 0) return hipSuccess;
  if (sh.MT != 2) return hipErrorInvalidValue;
  if (sh.op == OP_E) {
    if (sh.prec == PREC_FP32) return launch_encode_nt<OP_E, PREC_FP32>(sh, heldcoef, strmcoef, sdata, out_part, sens, L, G, stop, s);
    if (sh.prec == PREC_BF16) return launch_encode_nt<OP_E, PREC_BF16>(sh, heldcoef, strmcoef, sdata, out_part, sens, L, G, stop, s);
    return launch_encode_nt<OP_E, PREC_FP16>(sh, heldcoef, strmcoef, sdata, out_part, sens, L, G, stop, s);
  }
  if (sh.prec == PREC_FP32) return launch_encode_nt<OP_EH, PREC_FP32>(sh, heldcoef, strmcoef, sdata, out_part, sens, L, G, stop, s);
  if (sh.prec == PREC_BF16) return launch_encode_nt<OP_EH, PREC_BF16>(sh, heldcoef, strmcoef, sdata, out_part, sens, L, G, stop, s);
  return launch_encode_nt<OP_EH, PREC_FP16>(sh, heldcoef, strmcoef, sdata, out_part, sens, L, G, stop, s);
}

hipError_t launch_finish_E_to_m(const float* epart, int nsplit, int64_t HC16, int NB, int64_t K, int G,
                                const float* unscale, float2* m, hipStream_t s) {
  if (K * G == 0) return hipSuccess;
  hipLaunchKernelGGL(finish_E_to_m_kernel, grid1(K * G), dim3(256), 0, s, epart, nsplit, HC16, NB, K, G, unscale, m);
  return hipGetLastError();
}

hipError_t launch_finish_E_to_ybuf(const float* epart, int nsplit, int64_t HC16, int NB, const float* unscale,
                                   float* ybuf, const int* stop, hipStream_t s) {
  const int64_t n = HC16 * NB * 16;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(finish_E_to_ybuf_kernel, grid1(n), dim3(256), 0, s, epart, nsplit, n, unscale, ybuf, stop);
  return hipGetLastError();
}

hipError_t launch_finish_EH(const float2* hpart, int nsplit, int64_t HC16, int64_t L, const float* unscale,
                            float2* x, hipStream_t s) {
  if (L == 0) return hipSuccess;
  hipLaunchKernelGGL(finish_EH_kernel, grid1(L), dim3(256), 0, s, hpart, nsplit, HC16, L, unscale, x);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, grid1(n), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace nfs
