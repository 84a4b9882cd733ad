// Internal declarations shared by the kernel sources and the C ABI layer.
//
// Work decomposition of the encoding operator (gfx950, wave64):
//  * every contraction is "held" x "streamed": E holds samples (its output
//    rows) and streams voxels; E^H holds voxels and streams samples;
//  * items are grouped in chunks (tiles) of 16; a wave owns MT held tiles and
//    walks a contiguous range of streamed chunks;
//  * for each (held tile, streamed chunk) pair the wave builds the 16 x 16
//    phase tile phi = K_blk R_blk on the f16 matrix cores (coefficients
//    balanced per term and split into two f16 parts, NQ v_mfma 16x16x32
//    instructions), takes sin/cos of it in revolutions on the VALU and feeds
//    (cos, sin) straight into the complex contraction on the matrix cores
//    (16x16x32 f16/bf16, or 16x16x4 f32), against the packed data operand of
//    the streamed chunk;
//  * the streamed range can be split over several workgroups ("splits");
//    partial results are summed afterwards in a fixed order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nfs {

enum { OP_E = 0, OP_EH = 1 };
enum { PREC_FP32 = 0, PREC_BF16 = 1, PREC_FP16 = 2 };

constexpr int kChunk = 16;        // items per tile/chunk
constexpr int kWaves = 4;         // waves per workgroup in the encode kernels
constexpr int kCgBlocks = 256;    // max workgroups of the CG vector kernels
constexpr int kBmaxBlocks = 256;  // workgroups of the max-magnitude kernels
constexpr int kMaxTerms = 32;     // phase terms (t*b0 plus up to 31 field terms)
constexpr int kTmaxBlocks = 64;   // workgroups per side of the term-maxima kernel
// Largest phase bound (revolutions) for which the hardware sine and cosine
// take the phase directly; above it the argument is first reduced with
// v_fract.  The hardware range is +-256 revolutions; the margin covers the
// rounding of the bound itself.
constexpr float kRawPhaseBound = 128.f;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Sum of src[s * stride] over s = 0 .. n-1, added in that order (so rounded
// as the plain loop rounds it), with the loads of eight consecutive terms
// issued before their additions, so that they are in flight together
// instead of one memory latency each.
__device__ __forceinline__ float2 sum_strided(const float2* src, int n, int64_t stride) {
  float re = 0.f, im = 0.f;
  for (int s0 = 0; s0 < n; s0 += 8) {
    float2 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = s0 + k < n ? src[(int64_t)(s0 + k) * stride] : make_float2(0.f, 0.f);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (s0 + k < n) {
        re += v[k].x;
        im += v[k].y;
      }
  }
  return make_float2(re, im);
}

// phase MFMA instructions for P + 1 terms (t*b0 plus P field terms): three
// split products per term, 32 k-slots per instruction (1, 2 or 3)
inline int phase_instrs(int n_basis) { return (int)cdiv(3 * (n_basis + 1), 32); }
// held tiles per wave: 4 while the accumulators stay small (up to 16 coils),
// else 2 (the default; the autotuner may pick any valid count)
inline int held_tiles(int nb) { return nb <= 2 ? 4 : 2; }
// held-tile counts the encode kernel is built for: 2, and 4 up to 4 column
// blocks (8 blocks x 4 tiles would not fit the register file)
inline bool valid_held_tiles(int nb, int mt) { return mt == 2 || (mt == 4 && nb <= 4); }
// bytes of one packed phase chunk (16 items): NQ instructions x 64 lanes x 16 B
inline size_t phase_chunk_bytes(int nq) { return (size_t)nq * 64 * 16; }
// 16-column blocks for 2G real columns (re/im per coil), rounded to 1, 2, 4, 8
inline int col_blocks(int n_coil) {
  int nb = (int)cdiv(2 * n_coil, 16);
  if (nb <= 1) return 1;
  if (nb <= 2) return 2;
  if (nb <= 4) return 4;
  return 8;
}

// bytes of one packed data chunk (16 items) per column block: fp16 one
// 16-byte fragment per lane; bf16 and fp32 two (hi and lo parts)
inline size_t data_chunk_bytes(int prec) { return prec == PREC_FP16 ? 64 * 16 : 2 * 64 * 16; }
// FP16 and FP32 operands (f16 fragments) are scaled by powers of two
inline bool scaled_prec(int prec) { return prec != PREC_BF16; }

struct EncodeShape {
  int op;            // OP_E or OP_EH
  int prec;          // PREC_*
  int NQ, NB, MT;    // phase instructions, column blocks, held tiles per wave
  int64_t HC, SC;    // held / streamed chunk counts
  int nsplit;        // splits of the streamed range
  int64_t cps;       // streamed chunks per split
};

// One problem (slice) of a persistent encode launch: the arguments of its
// single-problem launch, its held-tile block count gx (the single launch's
// grid x), and the index of its first item in the launch's work list
// (items: gx * nsplit per slice, slices in list order; workgroups take
// items in list order from an atomic counter).
struct EncodeItem {
  const void* heldcoef;
  const void* strmcoef;
  const void* sdata;
  int64_t HC, SC, cps;
  float* out_part;
  const float2* sens;
  int64_t L;
  const unsigned* tmax;
  const int* stop;
  int64_t first;
  int G, T, NB, gx;
};
constexpr int kMaxBatchItems = 24;  // slices per persistent launch (the list is a kernel argument)
struct EncodeBatch {
  EncodeItem it[kMaxBatchItems];
  int n;
  int64_t total;  // items in the work list
  int* counter;   // next item to take (device int, zero at launch)
};
// Whether a persistent launch handles this operand form and shape
// (FP16 / BF16 operands, NQ <= 2, NB in {1, 2, 4}).
bool persistent_supported(int prec, int NQ, int NB, int MT);
// All slices of b in one launch of `grid` workgroups (same op, precision,
// NQ, NB and MT for every slice).
hipError_t launch_encode_persistent(int op, int prec, int NQ, int NB, int MT, const EncodeBatch& b, int grid,
                                    hipStream_t s);

// ---- launchers (encode_kernels.hip) ---------------------------------------
// per-term largest magnitudes of the phase coefficients, as float bits:
// tmax[b] = max_k |a_b(k)| (a_0 = t, a_{b+1} = kcoef[.][b], before the 1/2pi
// scaling), tmax[kMaxTerms + b] = max_l |h_b(l)| (h_0 = b0, h_{b+1} =
// fields[b]); clears tmax first
hipError_t launch_term_absmax(const float* t, const float* kcoef, int64_t K, const float* b0, const float* fields,
                              int64_t L, int P, unsigned* tmax, hipStream_t s);
// side 0: samples (c0 = t, cb = kcoef [K][P]); side 1: voxels (c0 = b0, cb = fields [P][L]);
// role 0: streamed side (MFMA operand A), role 1: held side (operand B)
hipError_t launch_pack_phase(const float* c0, const float* cb, int64_t n_items, int P, int side, int role, int NQ,
                             const unsigned* tmax, void* out, hipStream_t s);
hipError_t launch_scale_sens(const float2* sens, const float* icorr, int G, int64_t L, float2* out,
                             hipStream_t s);
// value(item, c) = src[item*is + c*cs] * (mul ? mul[c*n_items + item] : 1) * (wgt ? wgt[item] : 1)
hipError_t launch_absmax(const float2* src, const float2* mul, const float* wgt, int64_t n_items, int64_t is,
                         int64_t cs, int G, float* bmax, const int* stop, hipStream_t s);
hipError_t launch_pack_data(int op, int prec, const float2* src, const float2* mul, const float* wgt,
                            int64_t n_items, int64_t is, int64_t cs, int G, int NB, int64_t nchunks, void* out,
                            const float* bmax, float* unscale, const int* stop, hipStream_t s);
// tmax/T: the term maxima above and the term count P + 1 (phase range check)
hipError_t launch_encode(const EncodeShape& sh, const void* heldcoef, const void* strmcoef,
                         const void* sdata, float* out_part, const float2* sens, int64_t L, int G,
                         const unsigned* tmax, int T, const int* stop, hipStream_t s);
// resident P (FP16 only): build the (cos, sin) fragments of all held-tile x
// streamed-chunk pairs into P [HC][SC][64][8 f16], and contract against them
hipError_t launch_build_P(int NQ, const void* heldcoef, const void* strmcoef, int64_t HC, int64_t SC,
                          const unsigned* tmax, int T, void* P, hipStream_t s);
hipError_t launch_resident(const EncodeShape& sh, const void* P, const void* sdata, float* out_part,
                           const float2* sens, int64_t L, int G, const int* stop, hipStream_t s);
inline size_t resident_P_bytes(int64_t HC, int64_t SC) { return (size_t)HC * (size_t)SC * 64 * 16; }
// sum E partials -> m[G][K] (coil-major) times *unscale
hipError_t launch_finish_E_to_m(const float* epart, int nsplit, int64_t HC16, int NB, int64_t K, int G,
                                const float* unscale, float2* m, hipStream_t s);
// E^H data operand of the samples straight from the E partials (E^H E):
// value(k, c) = sum_s epart[s][k][2c] + i epart[s][k][2c+1]; for FP16 scaled
// by 2^-(ceil(log2 L) + 1) with *unscale_out = *unscale_in times the inverse
// wgt (per sample, or NULL) times wmul multiplies the E output first
hipError_t launch_pack_EH_from_epart(int prec, const float* epart, int nsplit, int64_t HC16, int NB, int64_t K, int G,
                                     int64_t L, const float* wgt, float wmul, const float* unscale_in,
                                     float* unscale_out, int64_t nchunks, void* out, const int* stop, hipStream_t s);
// sum E^H partials -> x[L] times *unscale
hipError_t launch_finish_EH(const float2* hpart, int nsplit, int64_t HC16, int64_t L,
                            const float* unscale, float2* x, hipStream_t s);
hipError_t launch_fill_zero(float* p, int64_t n_floats, hipStream_t s);
hipError_t launch_fill(float* p, int64_t n_floats, float v, hipStream_t s);
// backward: grad_b0 from E^H(t o G) partials; grad_kcoef[:, b] from E(h_b o rho) partials
hipError_t launch_grad_b0(const float2* hpart, int nsplit, int64_t HC16, int64_t L, const float* unscale,
                          const float2* rho, float* out, hipStream_t s);
hipError_t launch_grad_kcoef(const float* epart, int nsplit, int64_t HC16, int NB, const float* unscale,
                             const float2* grad_m, int64_t K, int G, int P, int b, float* out, hipStream_t s);

// ---- stopping-criteria instrumentation (quality_kernels.hip) ------------------
// mean SSIM of |imgs[i]| against |ref| for i < n_img into out[i] (float64);
// images [n_img][L] complex, L = nx ny nz (x fastest); needs nx, ny >= 11 and
// nz == 1 or nz >= 11
size_t ssim_workspace_bytes(int n_img, int nx, int ny, int nz);
hipError_t launch_ssim(const float2* imgs, int n_img, const float2* ref, int nx, int ny, int nz, double* out, void* ws,
                       hipStream_t s);

// ---- k-space filter (postproc_kernels.hip) ------------------------------------
// One DFT along one axis of an [outer][n][inner] complex array:
// out = scale * g * DFT_sign(in) with g = f (per element, in the array's
// index order; NULL for 1); n <= kMaxDftAxis.
constexpr int kMaxDftAxis = 2048;
hipError_t launch_dft_axis(const float2* in, float2* out, int64_t outer, int n, int64_t inner, int sign, float scale,
                           const float* f, hipStream_t s);
hipError_t launch_filter_scale(const float2* in, float2* out, const float* f, float scale, int64_t L, hipStream_t s);

// ---- phase-basis compression on the device (compress_kernels.hip) ----------
constexpr int kCmpBlocks = 256;  // workgroups of its voxel reductions
// doubles of scratch for launch_compress_basis (partials, eigenvectors, r*)
size_t compress_workspace_doubles(int64_t L, int P);
// the host compression's arithmetic on device arrays; tmax: term maxima of
// launch_term_absmax; ws: compress_workspace_doubles(L, P) doubles
hipError_t launch_compress_basis(const float* fields, const float* b0, const float* kcoef, const float* t, int64_t L,
                                 int64_t K, int P, double rel_tol, const unsigned* tmax, double* ws,
                                 float* fields_out, float* b0_out, float* kcoef_out, float* t_out, double* theta,
                                 int* n_basis_out, double* err_bound, hipStream_t s);

// ---- CG (cg_kernels.hip) -----------------------------------------------------
struct CgState {
  float2* r;        // [L]
  float2* p;        // [L]
  float2* q;        // [L]
  float2* b;        // [L] E^H m (kept for residual replacement)
  double* part;     // [4][kCgBlocks] per-block partial sums
  double* alpha;    // [n_iter + 2] alpha_n = r_n^H r_n
  double* scal;     // [4]: beta, d2, unused, unused
  double* hist;     // [n_iter + 1][3]
  int* info;        // [2]
  int* stop;        // [1]
  float2* V;        // [n_iter + 1][L] normalised residuals (re-orthogonalisation) or NULL
  float2* rn;       // [L] the updated residual before re-orthogonalisation, or NULL
  float2* iters;    // [n_iter + 1][L] every iterate rho_n (traced solves), or NULL
  const float* icorr;  // [L] intensity correction applied to stored iterates, or NULL
  double* rpart;    // [n_iter + 1][2][kCgBlocks] partial dot products v_j^H r
  const float* smax;  // [L] max_c |S[c][l]| (FP16 operands) or NULL
  float* bmax;        // [kBmaxBlocks] bound on the next E operand (with smax)
  int64_t L;
  int nblk;         // CG workgroups
};
constexpr int kMaxReorth = 2048;

// One slice of the lock-step batched solve as its batched vector kernels
// read it (device memory, written once per solve): the CG state and the
// arguments its single-slice launches take.
struct CgSlice {
  CgState st;
  const float2* hpart;    // E^H partials [nsplit][stride]
  const float* unscale;   // their 1/scale
  float2* rho;            // the iterate
  int64_t stride;
  int nsplit;
};
// One slice's operand packing in the batched solve: the arguments of
// pack_data (E operand) or of pack_EH_from_epart (E^H operand of E^H E).
struct PackSlice {
  const void* src;          // pack_data: float2 items; pack_EH_from_epart: the E partials (float)
  const float2* mul;        // pack_data: per (coil, item) factor or NULL
  const float* wgt;         // per-item weight or NULL
  void* out;                // packed operand
  const float* bmax;        // pack_data: [kBmaxBlocks] magnitude bound (scaled precisions)
  const float* unscale_in;  // pack_EH_from_epart: 1/scale of the E operand
  float* unscale;           // 1/scale of the packed operand
  const int* stop;
  int64_t n_items, is, cs;  // pack_data: items and strides; pack_EH_from_epart: samples (n_items)
  int64_t nchunks, HC16;
  float scale, wmul;        // pack_EH_from_epart
  int G, NB, nsplit;
};
hipError_t launch_store_slice_args(const CgSlice& cg, const PackSlice& pe, const PackSlice& ph, CgSlice* cg_out,
                                   PackSlice* pe_out, PackSlice* ph_out, hipStream_t s);
// the vector steps of one iteration for the n slices of sl at once (grid
// (max_nblk, rows, n)); arithmetic and sums as the single-slice launches
hipError_t launch_cg_beta_batched(const CgSlice* sl, int n, int max_nblk, hipStream_t s);
hipError_t launch_cg_update_batched(const CgSlice* sl, int n, int max_nblk, int it, int nv, hipStream_t s);
hipError_t launch_cg_reorth_apply_batched(const CgSlice* sl, int n, int max_nblk, int nv, bool from_rn,
                                          hipStream_t s);
hipError_t launch_cg_direction_batched(const CgSlice* sl, int n, int max_nblk, int it, int n_iter, double tol,
                                       hipStream_t s);
// pack_data (op OP_E) / pack_EH_from_epart for the n slices of sl at once
// (grid (max_blocks, n), max_blocks: the largest single-slice grid)
hipError_t launch_pack_data_E_batched(int prec, const PackSlice* sl, int n, int64_t max_blocks, hipStream_t s);
hipError_t launch_pack_EH_from_epart_batched(int prec, const PackSlice* sl, int n, int64_t max_blocks,
                                             hipStream_t s);
// the E^H-operand scale of pack_EH_from_epart for L voxels
float epart_pack_scale(int prec, int64_t L);
hipError_t launch_cg_reset(const CgState& st, hipStream_t s);
// smax[l] = max_c |S[c][l]|
hipError_t launch_sens_absmax(const float2* sens, int G, int64_t L, float* smax, hipStream_t s);
hipError_t launch_cg_norm_m(const CgState& st, const float2* m, int64_t n, hipStream_t s);
hipError_t launch_cg_init(const CgState& st, const float2* hpart, int nsplit, int64_t stride,
                          const float* unscale, float2* rho, int64_t L, hipStream_t s);
hipError_t launch_cg_start(const CgState& st, int n_iter, hipStream_t s);
hipError_t launch_cg_beta(const CgState& st, const float2* hpart, int nsplit, int64_t stride,
                          const float* unscale, int64_t L, hipStream_t s);
// nv > 0: the new r goes to st.rn, and the partial dot products of it with
// V[0..nv) to rpart (grid (nblk, ceil(nv / 4)))
hipError_t launch_cg_update(const CgState& st, float2* rho, int64_t L, int n, int nv, hipStream_t s);
// nv > 0: also the partial dot products of the new r with V[0..nv) (rpart)
hipError_t launch_cg_replace(const CgState& st, const float2* hpart, int nsplit, int64_t stride,
                             const float* unscale, int64_t L, int nv, hipStream_t s);
// p = r + (alpha'/alpha) p (and, with st.smax, the E operand bound into st.bmax)
hipError_t launch_cg_direction(const CgState& st, int64_t L, int n, int n_iter, double tol, hipStream_t s);
// V[j] = r / sqrt(alpha_j)
hipError_t launch_cg_store_v(const CgState& st, int j, hipStream_t s);
// r -= sum_{j < nv} (v_j^H r) v_j; partial r^H r -> part[1]
// r = src - sum_{j < nv} (v_j^H src) v_j from the partials in rpart, src = st.rn
// (from_rn) or st.r; partial r^H r -> part[1]
hipError_t launch_cg_reorth_apply(const CgState& st, int nv, bool from_rn, hipStream_t s);
hipError_t launch_cg_finish(const CgState& st, float2* rho, const float* icorr, int64_t L, hipStream_t s);
hipError_t launch_phase_shift(const float2* m, float2* out, const double* theta, int G, int64_t K, int sign,
                              hipStream_t s);


// ---- map estimation (sensitivity and B0 maps from prescan data) ----
constexpr int kMaxSvdCoils = 16;   // coils of the per-voxel SVD (one 16x16 matrix-core tile)
constexpr int kMaxFitEchoes = 64;  // echoes of the B0 fit
constexpr int kMgCoarseMax = 64;   // unknowns of the coarsest multigrid level (explicit inverse)
constexpr int kPcgChunk = 32;      // PCG iterations enqueued between two reads of the status flags
enum { MAP_SENS = 0, MAP_B0 = 1 };
// PCG status per right-hand side (0 = running), same codes as the CG solve
enum { PCG_TOL = 2, PCG_EXACT = 3, PCG_BREAKDOWN = 4 };

// Jacobi-preconditioned CG over nrhs float64 right-hand sides of length L
// (each stored with stride Lp), all in the caller's workspace.
struct PcgState {
  double* x;
  double* r;
  double* p[2];  // ping-pong: iteration n reads p[n & 1], writes p[(n & 1) ^ 1]
  double* q;
  double* z;     // multigrid output M^-1 r (NULL with the Jacobi preconditioner)
  double* dinv;  // [Lp] inverse diagonal (0 on rows without entries)
  double* part0;  // [nrhs][nblk] workgroup partials
  double* part1;
  double* rz;     // [nrhs] r.(D^-1 r)
  double* alpha;
  double* beta;
  double* bb;     // [nrhs] b.b
  double* rr;     // [nrhs] r.r of the last iteration
  int* iters;     // [nrhs] iterations run
  int* status;    // [nrhs] 0 running, else PCG_*
  int64_t L, Lp;
  int nblk;   // workgroups of the vector kernels (256 voxels each)
  int ntile;  // workgroups of the stencil kernels (z-marching tiles)
  int npart;  // stride of part0 / part1: max(nblk, ntile)
  int nrhs;
};
size_t pcg_state_bytes(int nrhs, int nx, int ny, int nz, bool with_z);
PcgState pcg_state(void* base, int nrhs, int nx, int ny, int nz, bool with_z);
// workspace of the multigrid hierarchy for nrhs right-hand sides on an nx x ny x nz grid
size_t mg_bytes(int nrhs, int nx, int ny, int nz);
// Solve the MAP_SENS / MAP_B0 normal equations for st.nrhs right-hand sides b
// [nrhs][Lp] into st.x with the NFS_PRECOND_* preconditioner (mg_ws: mg_bytes
// of workspace, multigrid only); synchronises the stream every kPcgChunk
// iterations.  status, iters: host [nrhs].
hipError_t pcg_solve(int op, int precond, const PcgState& st, void* mg_ws, const double* b, int nx, int ny, int nz,
                     const double* t, const double* w, double alpha, double tol, int max_iter, int* status,
                     int* iters, hipStream_t s);

// S^ [G][L] (complex float64) from prescan X [G][ne][L] (complex float32), G <= 16
hipError_t launch_sens_initial(const float2* X, int G, int ne, int64_t L, double2* shat, hipStream_t s);
// b [3G][Lp]: mT |S^|, mT Re(S^/|S^|), mT Im(S^/|S^|)
hipError_t launch_sens_rhs(const double2* shat, const float* mT, int G, int64_t L, int64_t Lp, double* b,
                           hipStream_t s);
// S [G][L] = x_mag * x_n / |x_n| from the smoothed components x [3G][Lp]; either output may be NULL
hipError_t launch_sens_combine(const double* x, int G, int64_t L, int64_t Lp, float2* s32, double2* s64,
                               hipStream_t s);
// B0^ (rad/s), beta, eps [L] from prescan X and sensitivities S [G][L], ne <= kMaxFitEchoes
hipError_t launch_b0_fit(const float2* X, const float2* S, int G, int ne, int64_t L, double dte, double* b0hat,
                         double* beta, double* eps, hipStream_t s);
hipError_t launch_b0_store(const double* x, int64_t L, float* b0, double* b064, hipStream_t s);
// weights t, w [L] and st.dinv of the MAP_SENS (masks) or MAP_B0 (eps) system
hipError_t launch_smooth_setup(int op, int nx, int ny, int nz, const float* mT, const float* mR, const double* eps,
                               double alpha, double* t, double* w, const PcgState& st, hipStream_t s);

}  // namespace nfs
