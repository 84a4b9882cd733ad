/*
 * nfs.h -- C ABI of the MI355X (gfx950) non-Fourier SENSE library.
 *
 * The library evaluates the encoding operator E of higher-order ("non-Fourier")
 * SENSE, its adjoint E^H, the normal operator E^H E, and solves
 * E^H E rho = E^H sigma with conjugate gradients, as defined in the paper's
 * Methods section ("Implementation of the higher-order SENSE reconstruction":
 * the signal-model equations P = exp(i K R), E p = P (S o (p 1^T)),
 * E^H sigma = (S* o (P^H Sigma)) 1, and the CG listings of the
 * reconstruction-algorithm figure).
 *
 * Model.  For voxel l (0 <= l < L), sample k (0 <= k < K) and coil c
 * (0 <= c < G), with P field-basis terms,
 *     phi(k, l)  = sum_{b<P} kcoef[k][b] * fields[b][l] + t[k] * b0[l]      (radians)
 *     (E rho)[c][k] = sum_l sens[c][l] * exp(+i phi(k, l)) * rho[l]
 *     (E^H m)[l]    = sum_c conj(sens[c][l]) * sum_k exp(-i phi(k, l)) * m[c][k]
 * kcoef holds the dynamic field terms k_b(t_k) and t the sample times
 * (columns of the paper's temporal basis K); fields holds the spatial basis
 * h_b(r_l) and b0 the off-resonance map in rad/s (rows of the spatial basis R).
 *
 * Conventions for every call.
 *  - Every array argument is a DEVICE pointer owned by the caller; the library
 *    never allocates, frees or retains device memory.  Scratch space is the
 *    caller's workspace `ws` of at least nfs_workspace_bytes() bytes,
 *    256-byte aligned; its contents on entry are ignored and on exit undefined.
 *  - Complex arrays are interleaved (re, im) float pairs (complex64), 8-byte
 *    aligned; real arrays are float32, 4-byte aligned.  Multi-index arrays are
 *    row-major, last index contiguous, with the shapes given in brackets.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *    is asynchronous: the call returns once the work is enqueued.  Inputs are
 *    read-only and must not alias outputs or the workspace.
 *  - Return value: NFS_OK, or a negative status.  All argument checks run on
 *    the host before anything is enqueued, so an error leaves every output
 *    untouched.  A failed launch returns NFS_EHIP; device faults surface at
 *    the caller's next synchronisation.  nfs_last_error() gives a message for
 *    the last non-OK status of the calling thread.
 *  - Limits: 1 <= G <= 64; 0 <= P <= 31; 0 <= L, K <= 2^26.
 */
#ifndef NFS_H
#define NFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum nfs_status {
  NFS_OK = 0,
  NFS_EINVAL = -1,       /* null pointer, bad enum, misaligned pointer, non-finite scalar */
  NFS_ESHAPE = -2,       /* size out of the supported range */
  NFS_EHIP = -3,         /* HIP runtime error (device query or launch) */
  NFS_EWORKSPACE = -4,   /* workspace missing, misaligned or too small */
  NFS_EUNSUPPORTED = -6  /* device is not gfx950 */
};

/* Operand precision of the two complex contractions (the phase is always
 * float32-grade and its sin/cos float32; accumulation is always float32).
 *  NFS_FP32: float32-grade: both operands split into two float16 parts and
 *            the three leading products taken on the f16 matrix cores (about
 *            2^-21 relative per product).
 *  NFS_BF16: bfloat16 (cos, sin) operand against a two-part bfloat16 data
 *            operand (round to nearest even).
 *  NFS_FP16: float16 operands.
 *  For NFS_FP32 and NFS_FP16 the data operand is scaled by a power of two
 *  chosen on the device (from its maximum magnitude or a bound on it) and
 *  unscaled after the contraction (exact).
 * The phase is computed in revolutions; inputs whose phase bound
 * sum_b max|kcoef_b|/2pi * max|fields_b| (with t and b0 as term 0) exceeds
 * 2^20 revolutions carry no fractional phase in float32 and are outside the
 * supported range (results are not meaningful there).                       */
enum nfs_precision { NFS_FP32 = 0, NFS_BF16 = 1, NFS_FP16 = 2 };

/* Operation selector for nfs_workspace_bytes. */
enum nfs_op { NFS_OP_E = 0, NFS_OP_EH = 1, NFS_OP_EHE = 2, NFS_OP_CG = 3, NFS_OP_CG_RESIDENT = 4 };

/* Values of info[1] written by nfs_cg_solve. */
enum nfs_cg_status {
  NFS_CG_MAXITER = 1,    /* ran n_iter iterations */
  NFS_CG_TOL = 2,        /* ||r_n|| <= tol * ||r_0|| */
  NFS_CG_EXACT = 3,      /* r_n^H r_n == 0 (includes E^H sigma == 0) */
  NFS_CG_BREAKDOWN = 4   /* p^H E^H E p <= 0 or a non-finite CG scalar */
};

/* The reconstruction problem: sizes and the model arrays (all device). */
typedef struct nfs_problem {
  int64_t n_vox;        /* L: number of voxels (entries of rho) */
  int64_t n_samp;       /* K: number of samples, all shots concatenated */
  int32_t n_coil;       /* G: number of receive coils */
  int32_t n_basis;      /* P: number of dynamic field terms */
  const float* sens;    /* [G][L] complex: S_c(r_l) (the paper's S, stored transposed) */
  const float* fields;  /* [P][L] real: h_b(r_l) (rows 2..P+1 of the spatial basis R) */
  const float* b0;      /* [L] real, rad/s: B0(r_l) (row 1 of R, gamma folded in) */
  const float* kcoef;   /* [K][P] real, rad: k_b(t_k) (columns 2..P+1 of K, row-major) */
  const float* t;       /* [K] real, s: t_k (column 1 of K) */
  const float* icorr;   /* [L] real or NULL: intensity correction j (used by nfs_cg_solve only) */
} nfs_problem;

typedef struct nfs_ctx nfs_ctx;

/* Bind a context to HIP device `device` (checks that it is gfx950 and reads
 * its compute-unit count, used to size launch grids).  The context holds no
 * device memory.  Returns NFS_EHIP if the device cannot be queried and
 * NFS_EUNSUPPORTED if it is not gfx950; *ctx is NULL on error.            */
int nfs_create(nfs_ctx** ctx, int device);
int nfs_destroy(nfs_ctx* ctx);

/* Workspace bytes needed by `op` (enum nfs_op) at `precision` for problem
 * sizes `prob` (only the sizes and whether icorr is NULL are read; array
 * pointers may be NULL here).  For NFS_OP_CG and NFS_OP_CG_RESIDENT the size
 * also depends on n_iter and reorth (both ignored for the other ops);
 * NFS_OP_CG_RESIDENT (nfs_cg_solve_resident) adds 2 K L x 4 bytes for the
 * resident P and takes only NFS_FP16 (NFS_EUNSUPPORTED otherwise).
 * Host-only; never touches the device.                                    */
int nfs_workspace_bytes(const nfs_ctx* ctx, const nfs_problem* prob, int op, int precision,
                        int n_iter, int reorth, size_t* bytes);

/* m = E rho (signal-model equation for E).  rho: [L] complex; m: [G][K]
 * complex (coil-major, the paper's Sigma transposed).                     */
int nfs_apply_E(nfs_ctx* ctx, const nfs_problem* prob, const float* rho, float* m,
                int precision, void* ws, size_t ws_bytes, void* stream);

/* x = E^H m (adjoint equation, evaluated as sum_c conj(S_c) o (P^H m_c)
 * without forming P^H).  m: [G][K] complex; x: [L] complex.               */
int nfs_apply_EH(nfs_ctx* ctx, const nfs_problem* prob, const float* m, float* x,
                 int precision, void* ws, size_t ws_bytes, void* stream);

/* q = E^H E p (the normal operator applied in each CG iteration).
 * p, q: [L] complex.                                                      */
int nfs_apply_EHE(nfs_ctx* ctx, const nfs_problem* prob, const float* p, float* q,
                  int precision, void* ws, size_t ws_bytes, void* stream);

/* Conjugate gradients on E^H E rho = E^H m (reconstruction-algorithm
 * figure): rho_0 = 0, r_0 = p_0 = E^H m, then per iteration q = E^H E p,
 * beta = Re p^H q, rho += (alpha/beta) p, r -= (alpha/beta) q,
 * alpha' = r^H r, p = r + (alpha'/alpha) p.  If prob->icorr is not NULL the
 * sensitivities are multiplied by j first and rho by j at the end.
 *   m:         [G][K] complex coil data (input)
 *   rho:       [L] complex (output; written even if the loop stops early)
 *   n_iter:    maximum number of iterations, >= 0
 *   tol:       0 = run n_iter iterations; > 0 = stop once ||r_n|| <= tol ||r_0||
 *   replace_every: 0 = never; k > 0 = every k iterations replace the
 *              recursive residual by E^H m - E^H E rho (one extra E^H E)
 *   reorth:    0 = plain recurrences (as printed); 1 = after each residual
 *              update, orthogonalise r against all earlier normalised
 *              residuals (classical Gram-Schmidt, float64 dot products).
 *              Identical iterates in exact arithmetic; keeps float32/float16
 *              runs on the exact-arithmetic trajectory on ill-conditioned
 *              problems.  Needs n_iter <= 2048 and (n_iter+1)*L complex of
 *              workspace.
 *   hist:      device double [n_iter+1][3] or NULL; row n holds ||r_n||,
 *              ||rho_n|| and ||m - E rho_n||^2 from the recurrence
 *              ||d_{n+1}||^2 = ||d_n||^2 - alpha^2/beta (rows past the
 *              last iteration are left untouched)
 *   info:      device int [2] or NULL: iterations done, enum nfs_cg_status
 * All CG scalars (dot products, alpha, beta, norms) are float64 on the
 * device; vectors are complex64; the host never synchronises.              */
int nfs_cg_solve(nfs_ctx* ctx, const nfs_problem* prob, const float* m, float* rho,
                 int n_iter, double tol, int replace_every, int reorth, int precision,
                 double* hist, int* info, void* ws, size_t ws_bytes, void* stream);

/* The same solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no workspace argument; the scratch lives in a device array of the library
 * (NFS_SCRATCH_BYTES per GPU, held from library load until the process
 * ends; its address per device is looked up once, by nfs_create).  Same
 * arguments, results and rules as nfs_cg_solve, which it shares its kernels
 * with (results are bit-identical to nfs_cg_solve with the same encode
 * shapes).  Allocates nothing: NFS_EWORKSPACE if the solve needs more than
 * NFS_SCRATCH_BYTES (nfs_workspace_bytes with NFS_OP_CG gives the need;
 * the 2D 128x128 / 16-coil / 60000-sample workload takes about 140 MB at
 * its tuned shapes).  Every call on one GPU uses that GPU's one scratch
 * array and leaves it in an undefined state; calls that overlap on one GPU
 * (different streams or host threads without ordering) race and give
 * undefined results.                                                      */
#define NFS_SCRATCH_BYTES (256u * 1024u * 1024u)
int nfs_cg_solve_noalloc(nfs_ctx* ctx, const nfs_problem* prob, const float* m, float* rho, int n_iter, double tol,
                         int replace_every, int reorth, int precision, double* hist, int* info, void* stream);

/* The same solve in the non-split form of the reconstruction figure (left
 * column): the phase factors P = exp(i phi) are built once per solve, as the
 * float16 (cos, sin) operand of the FP16 contraction (2 K L x 4 bytes of
 * workspace: one copy per direction), and every E and E^H of the solve
 * streams them from memory instead of rebuilding them.  Same arguments,
 * results and rules as nfs_cg_solve; precision must be NFS_FP16
 * (NFS_EUNSUPPORTED otherwise); workspace: NFS_OP_CG_RESIDENT.  Meant for
 * problems whose P fits in memory (2D slices); results agree with
 * nfs_cg_solve up to the order of float32 sums.                            */
int nfs_cg_solve_resident(nfs_ctx* ctx, const nfs_problem* prob, const float* m, float* rho, int n_iter,
                          double tol, int replace_every, int reorth, int precision, double* hist, int* info,
                          void* ws, size_t ws_bytes, void* stream);

/* Stopping-criteria instrumentation (the paper's study of the CG iteration
 * count: L-curve and SSIM over up to 250 iterations).
 *
 * nfs_cg_solve_traced: nfs_cg_solve that also stores every iterate:
 *   iterates: device [n_iter+1][L] complex; row n = rho_n (row 0 = 0), with
 *             the intensity correction applied as to the output; rows past
 *             the last iteration are left untouched.
 * Workspace: NFS_OP_CG.                                                    */
int nfs_cg_solve_traced(nfs_ctx* ctx, const nfs_problem* prob, const float* m, float* rho, int n_iter, double tol,
                        int replace_every, int reorth, int precision, double* hist, int* info, float* iterates,
                        void* ws, size_t ws_bytes, void* stream);

/* Mean SSIM (Wang, Bovik, Sheikh, Simoncelli 2004, as cited by the paper)
 * of the magnitude of each of n_img images against the magnitude of `ref`:
 * Gaussian window sigma 1.5 truncated to 11 taps per axis and normalised,
 * C1 = (0.01 D)^2, C2 = (0.03 D)^2 with D = max - min of |ref|, window-
 * weighted statistics without sample-size correction, averaged over the
 * window positions fully inside the image.  Float64 throughout.
 *   imgs: device [n_img][L] complex, ref: device [L] complex, L = nx ny nz,
 *         voxel index x + nx (y + ny z); nx, ny >= 11, nz == 1 (2D) or >= 11
 *   out:  device double [n_img]
 * Workspace: nfs_ssim_workspace_bytes (256-byte aligned).                 */
int nfs_ssim_workspace_bytes(int n_img, int nx, int ny, int nz, size_t* bytes);
int nfs_ssim(nfs_ctx* ctx, const float* imgs, int n_img, const float* ref, int nx, int ny, int nz, double* out,
             void* ws, size_t ws_bytes, void* stream);

/* Corner of the L-curve (log ||rho_n||, log ||d_n||) from a CG history:
 * HOST arrays.  hist: [n_rows][3] as written by the CG solves (||r_n||,
 * ||rho_n||, ||d_n||^2); rows whose ||rho_n|| or ||d_n||^2 is not positive
 * and finite are left out.  The curvature of an interior point is that of
 * the circle through it and its two neighbours (signed, counter-clockwise
 * positive); *corner = the row of largest curvature, or -1 with fewer than
 * three usable rows.  kappa: host double [n_rows] or NULL (NaN where
 * undefined).                                                              */
int nfs_lcurve_corner(const double* hist, int n_rows, int* corner, double* kappa);

/* k-space filter (Methods, "Computation of k-space filters"; last line of
 * both reconstruction listings): rho_f = IFFT(FFT(rho) o f) on an image grid
 * nx x ny x nz (voxel index x + nx (y + ny z)), f real [L] in the same index
 * order, bin (u, v, w) standing for the signed frequency u (if u < ceil(nx/2),
 * else u - nx) and so on, in cycles per field of view.  The DFT is applied
 * one axis at a time (float32 sums, twiddles from double precision): forward
 * passes, then f and 1/L, then inverse passes, L (nx + ny + nz) complex
 * multiply-adds per direction.  rho, out: device [L] complex (must not
 * alias); f: device float [L].  Each axis at most 2048 long (NFS_ESHAPE
 * otherwise).  Workspace: nfs_kspace_filter_workspace_bytes (L complex,
 * rounded up to 256 bytes; ctx is not read).                              */
int nfs_kspace_filter_workspace_bytes(const nfs_ctx* ctx, int nx, int ny, int nz, size_t* bytes);
int nfs_apply_kspace_filter(nfs_ctx* ctx, const float* rho, float* out, int nx, int ny, int nz, const float* f,
                            void* ws, size_t ws_bytes, void* stream);
/* The filter itself: f = 1 on the bins inside the convex hull of the K
 * first-order k-space positions kpos (HOST double [K][dim], cycles per field
 * of view), 0 elsewhere; bins on the hull count as inside.  Host
 * computation.  dim 2 (with nz 1): convex hull by Andrew's monotone chain,
 * then an edge test per bin.  dim 3: convex hull by quickhull (on the
 * positions joggled by at most 5e-10 of their largest coordinate, which
 * keeps the visible regions of nearly coplanar trajectory samples simple),
 * then per (x, y) column the z interval the face planes allow; NFS_EINVAL
 * if the positions span no volume.
 * mask: HOST uint8 [L]; *n_inside (may be NULL): number of bins set.      */
int nfs_kspace_filter_mask(const double* kpos, int64_t K, int dim, int nx, int ny, int nz, unsigned char* mask,
                           int64_t* n_inside);

/* Phase-basis compression (host computation on host arrays).  The phase of
 * the signal model, phi(k, l) = t[k] b0[l] + sum_p kcoef[k][p] fields[p][l]
 * (the encoding matrix as the product of the sample-side and voxel-side
 * coefficient matrices), is rewritten as
 *   phi(k, l) = theta[k] + t'[k] b0'[l] + sum_{p < P'} kcoef'[k][p] fields'[p][l]
 * with P' + 1 <= P + 1 terms: each voxel-side row is scaled by its term's
 * largest sample coefficient and centred (its mean goes into the per-sample
 * offset theta), and the centred rows are replaced by their leading
 * principal directions (double-precision Gram matrix, Jacobi eigenvectors),
 * as many as make
 *   max_l sum_b |residual_b(l)| <= rel_tol * sum_b max|a_b| max|h_b|,
 * which bounds |phi' - phi| at every (k, l) by that fraction of the phase
 * bound.  rel_tol 0 selects 2^-24.  A basis evaluated on a lower-
 * dimensional set (16 solid harmonics up to third order on one slice span
 * the 10 polynomials of degree <= 3 in two variables) loses its dependent
 * terms, so every tile phase takes fewer matrix-core products.
 * Since theta depends on the sample only, E^H E is unchanged; the original
 * operators follow from the compressed ones as
 *   E m = diag(exp(+i theta)) E' m,   E^H m = E'^H (diag(exp(-i theta)) m)
 * (nfs_phase_shift), so a CG solve of the compressed problem on data
 * exp(-i theta) m returns the solution of the original one.
 * Inputs: HOST float arrays laid out as in nfs_problem (fields [P][L], b0 [L],
 * kcoef [K][P], t [K]).  Outputs (HOST, caller-allocated at the input sizes):
 * fields_out rows 0..P'-1 of [P][L], b0_out [L], kcoef_out the first K P'
 * entries as [K][P'] (row-major, P' columns), t_out [K], theta [K] double
 * (rad), *n_basis_out = P', *err_bound (may be NULL) = the residual bound
 * reached (rad).  NFS_EINVAL for NULL or non-finite inputs or a negative
 * rel_tol, NFS_ESHAPE for sizes outside those of nfs_problem.  The outputs
 * go into an nfs_problem with n_basis P' and the original sens and icorr. */
int nfs_compress_basis(const float* fields, const float* b0, const float* kcoef, const float* t, int64_t L,
                       int64_t K, int P, double rel_tol, float* fields_out, float* b0_out, float* kcoef_out,
                       float* t_out, double* theta, int* n_basis_out, double* err_bound);

/* The same compression on the GPU, from the problem's DEVICE arrays
 * (prob->fields, b0, kcoef, t; sens and icorr are not read) into DEVICE
 * outputs, so that a new geometry (the field coefficients are measured per
 * scan) costs a few launches instead of host copies: identical steps in
 * double precision, sums over voxels formed per workgroup and added in
 * workgroup order, so results match nfs_compress_basis up to the order of
 * those sums.  Outputs sized for the largest P' = P: fields_out [P][L]
 * (rows 0..P'-1 written), kcoef_out [K][P] (the first K P' entries written,
 * as [K][P']), b0_out [L], t_out [K], theta [K] double; n_basis_out: device
 * int receiving P'; err_bound: device double or NULL.  P' is known on the
 * host only after synchronising (one int to read back before building the
 * compressed nfs_problem).  Non-finite inputs give undefined outputs (the
 * host call rejects them).  Workspace: nfs_compress_workspace_bytes
 * (256-byte aligned).  Asynchronous on `stream`.                          */
int nfs_compress_workspace_bytes(const nfs_problem* prob, size_t* bytes);
int nfs_compress_basis_device(nfs_ctx* ctx, const nfs_problem* prob, double rel_tol, float* fields_out,
                              float* b0_out, float* kcoef_out, float* t_out, double* theta, int* n_basis_out,
                              double* err_bound, void* ws, size_t ws_bytes, void* stream);

/* out[c][k] = m[c][k] exp(i sign theta[k]) for sign = +1 or -1 (the
 * per-sample offset of nfs_compress_basis), rotation in double precision.
 * m, out: DEVICE [G][K] complex (out == m allowed); theta: DEVICE [K]
 * double.  Launched on `stream`.                                          */
int nfs_phase_shift(nfs_ctx* ctx, const float* m, float* out, int n_coil, int64_t K, const double* theta, int sign,
                    void* stream);

/* Many independent reconstructions (slices with uneven L, K and G) solved
 * together: each slice runs exactly the nfs_cg_solve sequence (same kernels,
 * so each slice's result is bit-identical to its single solve), forked from
 * `stream` onto up to 8 library-owned streams (default priority; slices
 * assigned longest-first by L*K*G) and joined back, so the slices overlap
 * on the GPU.  n_iter, tol, replace_every, reorth and precision apply to all
 * slices.  m, rho: host arrays of n_slices device pointers (as for
 * nfs_cg_solve); hist, info: host arrays of device pointers, or NULL (and
 * individual entries may be NULL).  The workspace (256-byte aligned, at
 * least nfs_workspace_bytes_batched bytes) is split into one CG workspace
 * per slice (each nfs_workspace_bytes of that slice, rounded up to 256), a
 * 1 KiB block of work-list counters for the persistent form and that
 * form's per-slice launch arguments (192 * n_slices bytes, then twice
 * 128 * n_slices bytes, each rounded up to 256); 0 bytes for n_slices 0,
 * which returns NFS_OK without work.                                      */
int nfs_workspace_bytes_batched(const nfs_ctx* ctx, int n_slices, const nfs_problem* probs, int precision,
                                int n_iter, int reorth, size_t* bytes);
int nfs_cg_solve_batched(nfs_ctx* ctx, int n_slices, const nfs_problem* probs, const float* const* m,
                         float* const* rho, int n_iter, double tol, int replace_every, int reorth,
                         int precision, double* const* hist, int* const* info, void* ws, size_t ws_bytes,
                         void* stream);

/* Graph replay for repeated solves.  When on, nfs_cg_solve and
 * nfs_cg_solve_batched capture their whole launch sequence into a hipGraph
 * the first time they see a given set of pointers and parameters and
 * replay it (one hipGraphLaunch) on later identical calls.  Ignored while
 * the caller's stream is itself being captured and while kernel profiling
 * is on.  At most 32 graphs are kept per context: capturing a new one
 * beyond that destroys the least recently used (after waiting for its last
 * launch to finish), so callers that pass fresh buffers on every call do
 * not grow the cache without bound.  The rest live until nfs_destroy.
 * Default off.                                                            */
int nfs_set_graphs(nfs_ctx* ctx, int on);

/* How nfs_cg_solve_batched runs the slices (default NFS_BATCH_STREAMS).
 *  NFS_BATCH_STREAMS: each slice runs its own complete solve; slices are
 *      spread over 8 library streams (longest first) and joined, so the
 *      slices' kernels overlap freely.
 *  NFS_BATCH_PERSISTENT: all slices step through CG in lock-step; per
 *      iteration the E and the E^H contractions of every slice are one
 *      persistent launch per shape class (column blocks, held tiles),
 *      whose fixed grid walks a work list of all its slices' tile blocks
 *      (slices of different L and K in the same launch; the classes run
 *      side by side on the library streams); between them the operand
 *      packing and each CG vector step of all slices are one batched launch
 *      (each slice's workgroups and arithmetic as in its own solve; the
 *      setup and residual replacements fork per-slice kernels over the
 *      streams instead).  Used when every slice has FP16 or BF16 operands,
 *      at most 20 field terms and at most 32 coils; otherwise the call runs
 *      as NFS_BATCH_STREAMS.
 * Either way each slice's result is bit-identical to its nfs_cg_solve.     */
enum nfs_batch_mode { NFS_BATCH_STREAMS = 0, NFS_BATCH_PERSISTENT = 1 };
int nfs_set_batch_mode(nfs_ctx* ctx, int mode);

/* Tile-shape autotuning of the fused encode kernel (the kernel that builds
 * the phase tiles of the signal model, takes their sine/cosine and applies
 * them, for E and for E^H).  For this problem's shape class (L, K, G, P and
 * `precision`) it times every candidate shape on the caller's stream, with
 * the problem's own phase coefficients and realistic operands (E of
 * rho = 1 + i, then E^H of that output): held tiles per wave (2 or 4) and the
 * split count of the streamed range (targets of 1..48 workgroups per CU).
 * The fastest shape per direction is kept in `ctx` and used by every later
 * call on a problem of the same shape class; nfs_workspace_bytes then
 * reflects it, so query workspace sizes after tuning.  Results of a tuned
 * call differ from an untuned one only in the order of the split sums.
 * Synchronises the stream (host waits on events); fails with NFS_EINVAL
 * while the stream is being captured.  Workspace: nfs_tune_workspace_bytes
 * (256-byte aligned, contents undefined afterwards).                       */
int nfs_tune_workspace_bytes(const nfs_ctx* ctx, const nfs_problem* prob, int precision, size_t* bytes);
int nfs_autotune(nfs_ctx* ctx, const nfs_problem* prob, int precision, void* ws, size_t ws_bytes, void* stream);
/* Batch tuning.  The slices of nfs_cg_solve_batched run concurrently, so
 * the best shape of a slice inside the batch is not its best shape alone.
 * This times batch-wide candidates (held tiles 2 or 4 where a slice allows
 * it, and a target of 1/4 .. 4 workgroups per CU per slice from which each
 * slice derives its split counts) as concurrent E^H E passes over all
 * slices, forked and joined as the batched solve does, and keeps the
 * resulting per-slice shapes in `ctx` (replacing earlier entries of the same
 * shape classes).  Same synchronisation, capture and workspace rules as
 * nfs_autotune; workspace: nfs_tune_workspace_bytes_batched.              */
int nfs_tune_workspace_bytes_batched(const nfs_ctx* ctx, int n_slices, const nfs_problem* probs, int precision,
                                     size_t* bytes);
int nfs_autotune_batched(nfs_ctx* ctx, int n_slices, const nfs_problem* probs, int precision, void* ws,
                         size_t ws_bytes, void* stream);
/* The encode shape later calls will use for `op` (NFS_OP_E or NFS_OP_EH):
 * held tiles per wave and split count (tuned, else the default choice).    */
int nfs_tuned_shape(const nfs_ctx* ctx, const nfs_problem* prob, int precision, int op, int* held_tiles,
                    int* nsplit);
/* Pin the encode shape of `op` (NFS_OP_E or NFS_OP_EH) for this problem's
 * shape class, as if the autotuner had chosen it (for instance a shape found
 * by an earlier nfs_autotune and stored by the caller): held tiles per wave
 * (2, or 4 for up to four 16-column blocks, i.e. up to 32 coils) and split
 * count 1..64.  NFS_EINVAL for other values.  Results differ from another
 * shape's only in the order of the split sums.  Host-only.               */
int nfs_set_shape(nfs_ctx* ctx, const nfs_problem* prob, int precision, int op, int held_tiles, int nsplit);

/* Backward of m = E rho for a real loss L, for field-map and trajectory
 * refinement.  grad_m is dL/dm in PyTorch's convention for complex tensors
 * (for L = ||E rho - sigma||^2 it is 2 (E rho - sigma)).  Differentiating the
 * signal model's phase phi = K R (Methods, signal-model equations) gives
 *   grad_rho[l]      = (E^H grad_m)[l]
 *   grad_b0[l]       = Im(conj(rho[l]) (E^H (t o grad_m))[l])
 *   grad_kcoef[k][b] = Im(sum_c grad_m[c][k] conj((E (fields[b] o rho))[c][k]))
 * (the paper has no gradients; this is their derivation).  rho: [L]
 * complex; grad_m: [G][K] complex; grad_rho: [L] complex, grad_b0: [L]
 * real, grad_kcoef: [K][P] real -- each output may be NULL to skip it.
 * Cost: one E^H for grad_rho, one for grad_b0, one E per field term for
 * grad_kcoef.  Workspace: nfs_workspace_bytes(NFS_OP_EHE).                 */
int nfs_encode_backward(nfs_ctx* ctx, const nfs_problem* prob, const float* rho, const float* grad_m,
                        float* grad_rho, float* grad_b0, float* grad_kcoef, int precision,
                        void* ws, size_t ws_bytes, void* stream);

/* Kernel timing for benchmarks.  While enabled, every launch of the fused
 * encode kernel (the phase/sincos/contraction kernel of E and of E^H) made
 * through `ctx` is bracketed by two HIP events recorded on its launch
 * stream.  nfs_profile_read waits for the recorded events, returns the
 * number of launches and their summed event-to-event time in milliseconds
 * for `kind` (0 = E, 1 = E^H), and forgets them.  Host-side bookkeeping only;
 * HIP events are created on first use and kept by the context.            */
int nfs_profile_enable(nfs_ctx* ctx, int on);
int nfs_profile_read(nfs_ctx* ctx, int kind, int* count, double* total_ms);

/* ------------------------------------------------------------------------
 * Map estimation from multi-echo prescan data (Methods, "Computation of
 * sensitivity maps" and "Computation of B0 maps").  Float64 arithmetic.
 * Prescan images: imgs [G][n_echo][L] complex, coil c and echo n of voxel l
 * at imgs[(c n_echo + n) L + l]; grid nx x ny x nz (nz = 1 in 2D), voxel
 * index x + nx (y + ny z).  The two smoothing calls solve their normal
 * equations by preconditioned CG (float64 vectors and scalars, fixed-order
 * reductions, one CG per right-hand side; the paper suggests an incomplete-
 * Cholesky preconditioner, here Jacobi or multigrid, see nfs_precond) until
 * ||r|| <= tol ||b|| or max_iter iterations; they SYNCHRONISE the stream (every 32 iterations, to
 * read the convergence flags) and so must not be captured into a graph.
 * info: HOST int [2] or NULL: (largest iteration count over the right-hand
 * sides, status as enum nfs_cg_status: NFS_CG_TOL when all converged,
 * NFS_CG_EXACT when all right-hand sides were 0 or hit r == 0,
 * NFS_CG_MAXITER if any ran out, NFS_CG_BREAKDOWN if any broke down).     */
enum nfs_map_kind { NFS_MAP_SENS = 0, NFS_MAP_B0 = 1 };

/* Preconditioner of the smoothing solves.
 *  NFS_PRECOND_JACOBI: the inverse diagonal.
 *  NFS_PRECOND_MG:     one symmetric multigrid V-cycle: levels that halve
 *      every axis longer than 2 (coarse point I at fine point 2I) down to
 *      at most 64 unknowns, the same stencil on each level with its weights
 *      averaged by the interpolation weights and alpha divided by 16 (second
 *      differences) or 4 (first differences), multilinear prolongation,
 *      restriction by its transpose over 2^(axes halved), two damped Jacobi
 *      sweeps (weight 0.6) before and after the coarse correction, and the
 *      explicit inverse on the coarsest level.  Far fewer iterations on the
 *      poorly conditioned sensitivity system.                              */
enum nfs_precond { NFS_PRECOND_JACOBI = 0, NFS_PRECOND_MG = 1 };

/* Workspace bytes of nfs_sens_maps (kind NFS_MAP_SENS) or nfs_b0_map
 * (NFS_MAP_B0) for n_coil coils on an nx x ny x nz grid with preconditioner
 * precond.                                                                 */
int nfs_maps_workspace_bytes(int kind, int n_coil, int nx, int ny, int nz, int precond, size_t* bytes);

/* Initial sensitivities S^: per voxel the first left singular vector of the
 * n_coil x n_echo matrix of prescan values (rows coils, columns echoes),
 * computed as the dominant eigenvector of its Gram matrix on the float64
 * matrix cores, with the phase fixed so that its coil sum is real and
 * non-negative; voxels whose values are all zero get 0.  Where the two
 * largest singular values coincide the vector is not unique and any unit
 * vector of the top eigenspace may be returned.
 *   imgs: device complex [G][n_echo][L]; 1 <= G <= 16, 1 <= n_echo <= 1024
 *   shat: device complex float64 (interleaved double pairs) [G][L]
 * Needs no workspace; asynchronous.                                       */
int nfs_sens_initial(nfs_ctx* ctx, const float* imgs, int n_coil, int n_echo, int64_t n_vox, double* shat,
                     void* stream);

/* Sensitivity maps: S^ as above, then per coil the least-squares solution
 * of the sensitivity-smoothing equation, i.e. the normal equations
 *   (diag(M_T^2) + alpha sum_d D2_d^T diag(M_R^2) D2_d) s = M_T o s^
 * for s^ = |S^| and for the real and imaginary parts of S^/|S^| (0 where
 * S^ = 0), recombined as S = |S|_s n_s / |n_s| (0 where n_s = 0).  D2_d
 * has one row (x[i-1] - 2 x[i] + x[i+1]) per voxel i whose two neighbours
 * along axis d exist, weighted by M_R at i.  Rows of the system without
 * any entry (voxels neither in M_T nor reached by a penalty row) give 0.
 *   mask_T, mask_R: device float [L] (M_T, M_R; normally 0/1)
 *   alpha >= 0; tol >= 0; max_iter >= 0; precond: enum nfs_precond
 *   sens: device complex [G][L] or NULL; sens64: device complex float64
 *   [G][L] or NULL (not both NULL); shat: device complex float64 [G][L] to
 *   receive S^, or NULL (then S^ stays in the workspace); parts: device
 *   double [3G][L] to receive the three smoothed components (|S|_s per
 *   coil, then Re n_s, then Im n_s), or NULL
 * Workspace: nfs_maps_workspace_bytes(NFS_MAP_SENS, ...).                 */
int nfs_sens_maps(nfs_ctx* ctx, const float* imgs, int n_coil, int n_echo, const float* mask_T, const float* mask_R,
                  int nx, int ny, int nz, double alpha, double tol, int max_iter, int precond, float* sens,
                  double* sens64, double* shat, double* parts, int* info, void* ws, size_t ws_bytes, void* stream);

/* B0 map: the prescan echoes combined with the sensitivities,
 * c_n = sum_c conj(S_c) x_cn / sum_c |S_c|^2 (0 where the sum is 0), the
 * phase of c_n conj(c_0) (0 for n = 0) unwrapped along the echoes (a jump
 * of at least pi is taken modulo 2 pi into (-pi, pi]), the least-squares
 * fit phi_n = a n + beta mod(n, 2), B0^ = a / delta_te (rad/s) and eps =
 * the root mean square residual (the B0-fit equation); then the solution
 * of the B0-smoothing equation's normal equations
 *   (I + alpha sum_d D1_d^T diag(eps^2) D1_d) B0 = B0^,
 * D1_d with one row (x[i+1] - x[i]) per voxel i whose next neighbour along
 * axis d exists, weighted by eps at i.
 *   sens: device complex [G][L]; 1 <= G <= 64; 3 <= n_echo <= 64;
 *   delta_te > 0 (s); alpha, tol, max_iter as above
 *   b0: device float [L] or NULL; b064: device double [L] or NULL;
 *   fit: device double [3][L] (B0^, beta, eps) or NULL; at least one given.
 *   With b0 and b064 both NULL only the fit runs (info = (0, 0)).
 * Workspace: nfs_maps_workspace_bytes(NFS_MAP_B0, ...).                   */
int nfs_b0_map(nfs_ctx* ctx, const float* imgs, int n_coil, int n_echo, const float* sens, int nx, int ny, int nz,
               double delta_te, double alpha, double tol, int max_iter, int precond, float* b0, double* b064,
               double* fit, int* info, void* ws, size_t ws_bytes, void* stream);

/* Message for the last non-OK status returned on the calling thread. */
const char* nfs_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int nfs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NFS_H */
