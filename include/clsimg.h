/*
 * clsimg.h - constrained least-squares radio image formation on AMD Instinct
 * MI355X (gfx950).
 *
 * Method: A. Mouri Sardarabadi, A. Leshem, A.-J. van der Veen, "Radio
 * Astronomical Image Formation using Constrained Least Squares and Krylov
 * Subspaces".  One covariance snapshot (the paper's K = 1) per call.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Antenna p sits at (x_p, y_p) metres (planar array); `lambda` is the
 *    wavelength in metres.  Pixel i = im*nl + il of the grid looks towards
 *    direction cosines (l0 + il*dl, m0 + im*dm).
 *  - Array response (Sec. II-A normalisation, Sec. III-E model with z = 0):
 *        a_i[p] = P^-1/2 exp(-j 2 pi (x_p l_i + y_p m_i) / lambda).
 *  - Covariances are P x P complex64 matrices, row-major, R[p*P + q] =
 *    E{y_p conj(y_q)}; they must be Hermitian.  A transposed matrix mirrors
 *    the image.
 *  - Every large array is a DEVICE pointer on the context's device, owned by
 *    the caller; it must stay valid until the work queued on `stream`
 *    finishes.  Small descriptors (clsimg_array, clsimg_grid, clsimg_opts,
 *    clsimg_stats and the positions they point to) are HOST memory, read or
 *    written before the call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is ordered on it.  Calls that return results to the host
 *    (clsimg_solve's statistics, the active-set decisions) synchronise it.
 *  - One context per host thread and stream: a context is not thread safe.
 *  - Return value: CLSIMG_OK (0), a positive warning (results valid), or a
 *    negative error (outputs not written).  No C++ exception crosses the ABI.
 *  - Limits: 1 <= P <= CLSIMG_MAX_P, 1 <= nl*nm <= CLSIMG_MAX_Q.
 */
#ifndef CLSIMG_H
#define CLSIMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CLSIMG_MAX_P 288
#define CLSIMG_MAX_Q (1 << 20)

/* status codes */
#define CLSIMG_OK 0
#define CLSIMG_WMAXOUTER 1   /* active-set iteration limit reached; sigma is feasible   */
#define CLSIMG_WITNLIM 2     /* some LSQR subproblem hit its iteration limit             */
#define CLSIMG_WCYCLE 3      /* released pixel blocked again at zero step; state restored */
#define CLSIMG_EINVAL (-1)   /* NULL pointer, bad size, bad grid or option                */
#define CLSIMG_ENOTPD (-2)   /* covariance not positive definite or not finite           */
#define CLSIMG_ENOMEM (-3)   /* workspace would exceed the context's HBM budget          */
#define CLSIMG_EHIP (-4)     /* a HIP runtime call failed                                */
#define CLSIMG_ENOTSUP (-5)  /* option not available for this problem (see cost below)   */
#define CLSIMG_EWORKSPACE (-6) /* a device buffer a call needs was missing or too small */
                               /* (checked before any launch; an internal error)        */

/* bound kinds for clsimg_opts.bound */
#define CLSIMG_BOUND_MVDR 0  /* gamma = C / (a^H R^-1 a) (+ kappa_b std), Sec. II-D  */
#define CLSIMG_BOUND_MF 1    /* gamma = MF dirty image (+ kappa_b std), eq. mfupper  */
#define CLSIMG_BOUND_NONE 2  /* gamma = +inf: lower bound only, eq. NNLS             */

/* arithmetic of the full-grid beamforming products.  FP16 / BF16: the dirty
 * image and the bound take each operand split into high and low halves (three
 * 16x16x32 products accumulated in FP32, power-of-two scaling keeping FP16 in
 * range: close to FP32 results, about 2^-16 relative with BF16); the Lagrange
 * multipliers of each host-driven step take one half-precision product, and
 * the pixels its rounding bound cannot rule out are evaluated again in FP32,
 * so the release decision is the FP32 one.  The LSQR subproblems and the
 * device-resident loop (P <= 48) compute in FP32 in every mode, the Cholesky
 * factorisation and the LSQR scalars in FP64. */
#define CLSIMG_FP32 0  /* FP32 MFMA (16x16x4)                                         */
#define CLSIMG_FP16 1  /* FP16 MFMA (16x16x32) with FP32 accumulation                 */
#define CLSIMG_BF16 2  /* BF16 MFMA (16x16x32) with FP32 accumulation                 */

/* cost function for clsimg_opts.cost */
#define CLSIMG_COST_LS 0     /* 1/2 ||B0 - Psi sigma||^2, eq. CLS                         */
#define CLSIMG_COST_PWLS 1   /* preconditioned weighted LS, eq. preWLS: R^-1/2 weighting  */
                             /* on both sides, variable D sigma with D_i = h_i^2 / C,     */
                             /* h_i = a_i^H R^-1 a_i; threshold kappa_d std of the MVDR   */
                             /* image (App. A).  Needs P <= 96 (CLSIMG_ENOTSUP beyond):    */
                             /* the device-resident loop up to 48, the host-driven loop   */
                             /* (whitened steering rows of the free set) beyond, or when  */
                             /* the free set outgrows one workgroup.                      */

/* loop driving the Table I iteration (clsimg_opts.loop); both give the same
 * iterates and results */
#define CLSIMG_LOOP_AUTO 0   /* on the device for P <= 48 (continued on the host if the  */
                             /* free set outgrows one workgroup), host-driven beyond     */
#define CLSIMG_LOOP_HOST 1   /* host-driven for every P (measurement, tests)             */

/* LSQR engine of the host-driven loop (clsimg_opts.lsqr_engine); every engine
 * computes the same iterates, an engine that does not fit the problem falls
 * back to the next one down the list */
#define CLSIMG_LSQR_AUTO 0        /* the first that fits, in the order below; above 48 */
                                  /* antennas the two-kernel step before the cooperative */
                                  /* kernel (the faster there)                           */
#define CLSIMG_LSQR_ONE_WG 1      /* one workgroup, free set in LDS (P <= 48)            */
#define CLSIMG_LSQR_COOP 2        /* one cooperative multi-workgroup kernel (P <= 64)    */
#define CLSIMG_LSQR_TWO_KERNEL 3  /* two kernels per LSQR step (P <= 96); beyond, the    */
                                  /* correlation with separate reductions and adjoint    */

/* pixel states in clsimg_solve's `state` output */
#define CLSIMG_STATE_L 0     /* sigma_i = 0        */
#define CLSIMG_STATE_F 1     /* 0 < sigma_i < gamma_i (free)          */
#define CLSIMG_STATE_U 2     /* sigma_i = gamma_i  */

typedef struct clsimg_ctx clsimg_ctx;

/* layout-compatible with torch.complex64 / std::complex<float> */
typedef struct {
  float re, im;
} clsimg_c32;

typedef struct {
  int32_t P;              /* number of antennas                                */
  const double* pos_xy;   /* HOST, P x 2 row-major (x_p, y_p), metres          */
  double lambda;          /* wavelength, metres                                */
} clsimg_array;

typedef struct {
  int32_t nl, nm;         /* pixels along l and m; Q = nl*nm                   */
  double l0, dl, m0, dm;  /* first direction cosine and step along each axis   */
} clsimg_grid;

typedef struct {
  int32_t bound;          /* CLSIMG_BOUND_*                          (MVDR)     */
  double C;               /* MVDR bias factor, App. A gives N/(N-P)  (1.0)      */
  double kappa_b;         /* bound inflation in std units, App. A    (0.0)      */
  double kappa_d;         /* detection threshold in std units, Sec. III-C (6.0) */
  int64_t nsamples;       /* N samples behind R, used by eps and kappa_b        */
  double atol, btol;      /* LSQR tolerances                         (1e-6)     */
  double conlim;          /* LSQR condition limit                    (1e8)      */
  int32_t itnlim;         /* LSQR iterations per subproblem, -1 = 4|F|+100      */
  int32_t max_outer;      /* subproblem solves, -1 = 4Q                         */
  int32_t precision;      /* CLSIMG_FP32 | CLSIMG_FP16 | CLSIMG_BF16            */
  int32_t cost;           /* CLSIMG_COST_*                           (LS)       */
  int32_t loop;           /* CLSIMG_LOOP_*                           (AUTO)     */
  int32_t lsqr_engine;    /* CLSIMG_LSQR_* of the host-driven loop   (AUTO)     */
  int32_t hand_over_free; /* device loop, batches and server slots: continue on */
                          /* the host once |F| exceeds this; 0 = only when F    */
                          /* outgrows one workgroup                   (0)       */
  int32_t trace;          /* 1: host-driven loop with one line per Table I step */
                          /* on stderr                                (0)       */
  int32_t batch_graph;    /* clsimg_solve_batch: 1 replays each round's step    */
                          /* launches from a captured HIP graph, 0 enqueues     */
                          /* them one by one (same results)           (0)       */
} clsimg_opts;

typedef struct {
  int32_t status;
  int32_t outer_iters;    /* subproblem solves (Table I image index)            */
  int32_t adds;           /* pixels released into the free set                  */
  int32_t drops;          /* pixels blocked at a bound                          */
  int32_t lsqr_iters_total;
  int32_t lsqr_itnlim_hits;
  int32_t nF, nU;         /* final set sizes                                    */
  double rel_residual;    /* ||B0 - Psi sigma||_F / ||B0||_F at the final image; with */
                          /* CLSIMG_COST_PWLS the whitened residual of eq. preWLS,   */
                          /* ||L^-1 (B0 - Psi sigma) L^-H||_F / ||L^-1 B0 L^-H||_F   */
  double objective;       /* 1/2 the squared residual norm (numerator above)        */
  double min_margin_lambda; /* min |lambda_i + eps_i| / eps_i over detection tests */
  double min_margin_z;      /* min over accepted subproblems of min(z, gamma-z)/gamma */
  double psi_flops;         /* dense-count flops of every Psi / Psi^H applied: 8 P^2 per pixel
                               and correlation term, + 8 P per beamformed pixel             */
} clsimg_stats;

/* Fill `opts` with the defaults listed above (nsamples = 0: must be set). */
void clsimg_default_opts(clsimg_opts* opts);

/* Create a context on HIP device `device`.  `hbm_budget_bytes` caps the
 * workspace the context may allocate (0 = no cap).  The context owns that
 * workspace and caches the steering tables of the last (array, grid). */
int clsimg_create(clsimg_ctx** ctx, int32_t device, size_t hbm_budget_bytes);

/* Release the context and its workspace (synchronises its device). */
int clsimg_destroy(clsimg_ctx* ctx);

/* Matched-filter dirty image, eq. mfdimg at K = 1:
 *   mf[i] = a_i^H R a_i,  i = 0..Q-1.
 * R: DEVICE complex64 P x P.  precision: CLSIMG_FP32 / _FP16 / _BF16.
 * mf: DEVICE float[Q]. */
int clsimg_dirty_image(clsimg_ctx* ctx, const clsimg_c32* R, const clsimg_array* array,
                       const clsimg_grid* grid, int32_t precision, float* mf, void* stream);

/* The same dirty image with the device's own timestamps of its kernels, for
 * measuring the beamformer without the launch gaps around it: the start of the
 * first kernel is recorded into `start_event` and the end of the last kernel
 * into `stop_event` (hipEvent_t handles created by the caller with timing
 * enabled, passed as void*), so that hipEventElapsedTime(start, stop) is the
 * kernels' device time.  Both events must be non-null.  Arrays above
 * CLSIMG_MAX_P antennas (no full-grid beamformer) return CLSIMG_ENOTSUP. */
int clsimg_dirty_image_timed(clsimg_ctx* ctx, const clsimg_c32* R, const clsimg_array* array,
                             const clsimg_grid* grid, int32_t precision, float* mf, void* start_event,
                             void* stop_event, void* stream);

/* The dirty image of clsimg_dirty_image (same kernels, same bits) without
 * any allocation, for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Its workspace (antenna positions, steering tables, fragments of R: at most
 * 8 MiB) is a static array of the library that every GPU holds once, until
 * the process ends; ctx (created beforehand, outside the caller's
 * allocation-free region) holds this device's address of it.  The call
 * allocates nothing and does not touch the context's own workspace; the
 * positions are copied from host memory on `stream`.  Calls on one GPU share
 * that array: calls that overlap on one GPU (other streams, other contexts
 * or threads) race and must be ordered by the caller.  Arguments as
 * clsimg_dirty_image; CLSIMG_ENOMEM when the geometry needs more than the
 * 8 MiB (steering tables of Pp (nl + nm) entries, Pp = P rounded up to a
 * multiple of 8, plus the fragments of R beyond 48 antennas). */
int clsimg_dirty_image_noalloc(clsimg_ctx* ctx, const clsimg_c32* R, const clsimg_array* array,
                               const clsimg_grid* grid, int32_t precision, float* mf, void* stream);

/* Autotuner of the GEMM-shaped full-grid beamformers (the dirty image, bound
 * and multipliers for P > 48 in FP32, and for every P in split FP16 / BF16):
 * times one dirty image of this array and grid for each candidate number of
 * 16-pixel tiles per workgroup (2, 4, 8) on `stream`, and keeps the fastest in
 * the context for this precision and array size (by row tiles per wave,
 * ceil(P / 32); the last tuning of a size applies to every grid).  Every
 * candidate computes each pixel with the same operations in the same order,
 * so results are bit-identical whichever is kept.  Eight tiles are offered up
 * to P = 192 in FP32 (beyond, the accumulators would not fit in registers) and
 * up to P = 128 in split FP16 / BF16 (beyond, a block's operands would not fit
 * in LDS).  Not
 * for use under stream capture: it synchronises the stream.  chosen (host, may
 * be null): the tile count kept.  us (host float[3], may be null): microseconds
 * per dirty image for 2, 4 and 8 tiles (-1: not offered).  CLSIMG_ENOTSUP for FP32 with P <= 48 (the
 * register-resident beamformer has no tile choice) and for P > CLSIMG_MAX_P. */
int clsimg_autotune(clsimg_ctx* ctx, const clsimg_array* array, const clsimg_grid* grid, int32_t precision,
                    int32_t* chosen, float* us, void* stream);

/* Sets the tiles per workgroup of the GEMM-shaped beamformers for arrays of P
 * antennas at `precision` (tiles 2, 4, or 8 up to P = 192 in FP32 and up to
 * P = 128 in FP16 / BF16; 0 restores the built-in default), e.g. to reuse a
 * choice tuned earlier.  CLSIMG_EINVAL for other values. */
int clsimg_set_beam_tiles(clsimg_ctx* ctx, int32_t P, int32_t precision, int32_t tiles);

/* Device time of the full-grid multiplier kernel of the host-driven active-set
 * loop (the gradient of every feasible Table I step, eq. gls: beam_big_kernel
 * in FP32, the single half-precision product beam_h1_kernel with FP16 / BF16),
 * for measurement: while enabled, clsimg_solve binds two HIP events to each
 * such launch and adds their elapsed time after the step's read-back.  Writes
 * the milliseconds and launch count accumulated since the previous call
 * (host pointers, may be null), resets them, and sets the mode (enable != 0)
 * for later solves.  The device-resident loop (P <= 48) is not timed. */
int clsimg_kernel_timing(clsimg_ctx* ctx, int32_t enable, double* ms, int32_t* launches);

/* Upper bound gamma of the box constraint (eq. CLS):
 *   MVDR (eq. wmvdr, Sec. II-D): h_i = a_i^H R^-1 a_i with R = L L^H factored in
 *        FP64 on the device; gamma_i = C/h_i + kappa_b / (h_i sqrt(N-P-1));
 *   MF:  gamma_i = mf_i (1 + kappa_b / sqrt(N))   (App. A variance, K = 1);
 *   NONE: gamma_i = +inf.
 * Fails with CLSIMG_ENOTPD when the Cholesky factorisation breaks down.
 * R: DEVICE complex64 P x P.  gamma: DEVICE float[Q]. */
int clsimg_mvdr_bound(clsimg_ctx* ctx, const clsimg_c32* R, const clsimg_array* array,
                      const clsimg_grid* grid, const clsimg_opts* opts, float* gamma,
                      void* stream);

/* Correlation (forward) operator of Sec. IV-B on a pixel subset S:
 *   Y = sum_k v[k] a_{idx[k]} a_{idx[k]}^H     (= Psi_S v as a P x P matrix).
 * idx: DEVICE int32[n] pixel indices in [0, Q) (NULL = pixels 0..n-1);
 * v: DEVICE float[n]; Y: DEVICE complex64 P x P (overwritten; zero if n = 0). */
int clsimg_forward(clsimg_ctx* ctx, const clsimg_array* array, const clsimg_grid* grid,
                   const int32_t* idx, const float* v, int32_t n, clsimg_c32* Y, void* stream);

/* Beamforming (adjoint) operator of Sec. IV-B on a pixel subset S:
 *   g[k] = Re(a_{idx[k]}^H U a_{idx[k]})        (= Psi_S^H vect(U), real part).
 * U: DEVICE complex64 P x P Hermitian; idx: DEVICE int32[n] in [0, Q)
 * (NULL = pixels 0..n-1); g: DEVICE float[n]. */
int clsimg_adjoint(clsimg_ctx* ctx, const clsimg_array* array, const clsimg_grid* grid,
                   const clsimg_c32* U, const int32_t* idx, int32_t n, float* g, void* stream);

/* Box-constrained LS image (eq. CLS with K = 1) by the active-set method of
 * Sec. III-C / Table I, each equality-constrained subproblem (eqs.
 * subproblemLS, bsubproblemLS) solved matrix-free by LSQR (Sec. IV).
 *   data  B0 = R - diag(noise_diag)           (noise_diag NULL: no noise term)
 *   bound gamma as clsimg_mvdr_bound; threshold eps_i = kappa_d mf_i / sqrt(N)
 * R: DEVICE complex64 P x P.  noise_diag: DEVICE float[P] or NULL.
 * sigma0 / state0: DEVICE float[Q] / uint8[Q] feasible starting image and its
 *   sets (both NULL = start from sigma = 0, every pixel in L; state0 values
 *   other than CLSIMG_STATE_F and CLSIMG_STATE_U read as L).
 * sigma: DEVICE float[Q] out.  state: DEVICE uint8[Q] out (CLSIMG_STATE_*).
 * mf, gamma: DEVICE float[Q] out, or NULL.  stats: HOST, always written.
 * Synchronises `stream` (the active-set decisions are read on the host). */
int clsimg_solve(clsimg_ctx* ctx, const clsimg_c32* R, const clsimg_array* array,
                 const clsimg_grid* grid, const float* noise_diag, const clsimg_opts* opts,
                 const float* sigma0, const uint8_t* state0, float* sigma, uint8_t* state,
                 float* mf, float* gamma, clsimg_stats* stats, void* stream);

/* One request of a batched solve or of a server. */
typedef struct {
  const clsimg_c32* R;      /* DEVICE, P x P sample covariance of this request       */
  clsimg_array array;       /* antenna positions and wavelength (P equal in a batch) */
  clsimg_grid grid;         /* pixel grid of this request                           */
  const float* noise_diag;  /* DEVICE, P, or NULL                                    */
  float* sigma;             /* DEVICE, Q: image (output)                             */
  uint8_t* state;           /* DEVICE, Q: CLSIMG_STATE_* (output)                    */
  float* mf;                /* DEVICE, Q, or NULL: MF dirty image (output)           */
  float* gamma;             /* DEVICE, Q, or NULL: upper bound (output)              */
  clsimg_stats stats;       /* HOST: statistics of this request (output); status is  */
                            /* the request's own code                                */
} clsimg_request;

/* Batched solve (Sec. III, Table I, with LSQR of Sec. IV-A) of n independent
 * imaging problems -- frequency channels, time slices, observations -- with
 * the same options.  Requests with different antenna counts run as one batch
 * per count, in order of first appearance.  For P <= 48 every outer step of
 * all requests runs in one kernel launch (one workgroup per request) and the
 * Lagrange multipliers of all requests in another, so the requests share the
 * GPU instead of queueing; each request's result is identical to what
 * clsimg_solve returns for it alone.  Each request may have its own array,
 * wavelength and grid.  With the least-squares cost and the MVDR bound in
 * FP32, the set-up of all requests (R^-1, steering tables, initial state,
 * dirty images and bounds) also runs as a few batched launches.  When every
 * request has the same array and grid, they all read one copy of the
 * steering tables.  A request whose free set outgrows one workgroup (or
 * passes hand_over_free) is then solved again alone, as clsimg_solve does
 * (the device loop hands it to the host-driven loop at the same step).
 * Beyond 48 antennas the requests are solved one after another on the
 * host-driven loop.  Either way each result is that of the request's solve
 * alone.  Returns CLSIMG_OK when every request ended with CLSIMG_OK, its
 * first negative code if a request failed, else the largest warning code;
 * per-request codes are in reqs[i].stats.status.  `reqs` is host memory
 * (n entries); n >= 1. */
int clsimg_solve_batch(clsimg_ctx* ctx, int32_t n, clsimg_request* reqs, const clsimg_opts* opts, void* stream);

/* ---- K covariance blocks over one pixel grid ---------------------------
 * Snapshots under the Earth's rotation (short-term integrations k whose
 * antenna positions are rotated, Q_k in the data model of Sec. II) or
 * frequency channels with the same sky (another wavelength): the stacked
 * data model of eq. vectRtotal / eq. blockdiagtilde. */
#define CLSIMG_MAX_BLOCKS 64

typedef struct {
  const clsimg_c32* R;      /* DEVICE, P x P sample covariance of this block     */
  clsimg_array array;       /* antenna positions of this block and wavelength    */
  const float* noise_diag;  /* DEVICE, P, or NULL                                 */
} clsimg_block;

/* Active-set solve (Sec. III, Table I, LSQR of Sec. IV-A) of the K-block
 * problem  min 1/(2K) sum_k ||R_k - diag(noise_k) - A_k diag(sigma) A_k^H||^2
 * s.t. 0 <= sigma <= gamma (eq. UCLS with the box of eq. CLS), all blocks
 * with the same P and the same options, on one grid:
 *   mf[i]    = (1/K) sum_k a_{i,k}^H R_k a_{i,k}                  (eq. mfdimg)
 *   gamma[i] = C K / sum_k h_{i,k} (+ kappa_b std, App. A), h = a^H R^-1 a
 *              (eq. wmvdr); CLSIMG_BOUND_MF: mf + kappa_b std; _NONE: inf
 *   eps[i]   = kappa_d sqrt(sum_k (a_{i,k}^H R_k a_{i,k})^2) / (K sqrt N)
 *   gradient (1/K) sum_k vectdiag(A_k^H E_k A_k) for the release test.
 * 1 <= K <= CLSIMG_MAX_BLOCKS; blocks: HOST array of K.  LS cost only
 * (CLSIMG_COST_PWLS: CLSIMG_ENOTSUP).  Outputs and stats as clsimg_solve
 * (sigma0/state0 are not taken: the solve starts from sigma = 0); stats
 * rel_residual is over all blocks and objective is the cost above.
 * Synchronises `stream`.  With K = 1 it solves the clsimg_solve problem on
 * the host-driven loop. */
int clsimg_solve_multi(clsimg_ctx* ctx, int32_t K, const clsimg_block* blocks, const clsimg_grid* grid,
                       const clsimg_opts* opts, float* sigma, uint8_t* state, float* mf, float* gamma,
                       clsimg_stats* stats, void* stream);

/* ---- Strong off-grid sources (Sec. III-E, eq. doals) --------------------
 * The subproblem on the free set F becomes
 *   min over (delta_F, sigma_F)  1/2 || b - Psi(delta)_F sigma_F ||^2,
 *   |delta_i,l| <= |dl|/2, |delta_i,m| <= |dm|/2,
 * pixel i's steering vector taken at its centre shifted by delta_i (direction
 * cosines).  Each subproblem runs `rounds` rounds of (LSQR for sigma_F at the
 * current offsets, one Gauss-Newton step per free pixel's offset, inter-pixel
 * coupling neglected, clipped to the pixel), then a final LSQR.  A pixel
 * enters F at its centre and its offset is reset when it leaves F; free
 * pixels' bounds are the bound formula at their shifted directions; the
 * upper set keeps on-grid steering and bounds; release tests and the gradient
 * on the active pixels stay on the grid.  offsets: DEVICE float[2Q] out,
 * (delta_l, delta_m) per pixel, zero outside F; sigma holds the powers at the
 * shifted positions.  0 <= rounds <= 16 (0: the plain subproblem, with the
 * free steering vectors formed directly in FP64 rather than from the tables).
 * P <= 96 and the LS cost; LSQR in one workgroup, or for free sets beyond
 * its LDS in one cooperative kernel (CLSIMG_ENOTSUP where neither holds the
 * free set).  Other arguments as clsimg_solve (no starting image);
 * synchronises `stream`. */
int clsimg_solve_offgrid(clsimg_ctx* ctx, const clsimg_c32* R, const clsimg_array* array, const clsimg_grid* grid,
                         const float* noise_diag, const clsimg_opts* opts, int32_t rounds, float* sigma,
                         uint8_t* state, float* offsets, float* mf, float* gamma, clsimg_stats* stats,
                         void* stream);

/* ---- Serving: continuous batching of independent requests -------------
 * A server solves a stream of imaging requests (Sec. III, Table I, LSQR of
 * Sec. IV-A), each with its own array (any P <= CLSIMG_MAX_P), wavelength and
 * grid, all with the server's options.  Requests with P <= 48 are admitted
 * into device slots (at most max_slots, their device state in one arena of
 * hbm_budget_bytes, 0 = 1 GiB) as slots and arena space free up; each poll
 * runs steps_per_poll Table I steps of every admitted request, one kernel
 * launch per array tile-count group and step, and retires finished requests.
 * Other requests (larger P, or a free set beyond the device loop's on-chip
 * capacity) are solved by worker threads on streams of their own on the same
 * device, overlapping with the batch.  Every request's outputs equal those of
 * clsimg_solve for it alone.  The server owns one context and stream for the
 * batch, one per worker, the arena and the worker threads; submit / poll / query / destroy must be called from
 * one host thread.  With CLSIMG_COST_PWLS the workers' solves take P <= 96
 * (beyond, the request completes with status CLSIMG_ENOTSUP, as clsimg_solve). */
typedef struct clsimg_server clsimg_server;

typedef struct {
  int32_t pending;        /* submitted, waiting for a slot / arena space        */
  int32_t active;         /* in device slots                                    */
  int32_t worker_queued;  /* queued for, or being solved by, the worker         */
  int32_t ready;          /* finished, not yet returned by clsimg_server_poll   */
  int64_t submitted, admitted, completed;  /* completed = returned by poll       */
  int64_t step_rounds;    /* Table I steps launched for the device slots        */
  size_t arena_bytes, arena_used, arena_peak;
} clsimg_server_info;

/* Create a server on `device`.  1 <= max_slots <= 1024; 1 <= steps_per_poll
 * <= 1024 (steps between two looks at the requests' states: fewer give earlier
 * admission and retirement, more give fewer host round trips); 1 <= workers
 * <= 8 threads for the requests outside the device loop, each with its own
 * context and stream.  opts is copied.
 * Errors: CLSIMG_EINVAL, CLSIMG_ENOMEM (arena), CLSIMG_EHIP. */
int clsimg_server_create(clsimg_server** srv, int32_t device, int32_t max_slots, size_t hbm_budget_bytes,
                         int32_t steps_per_poll, int32_t workers, const clsimg_opts* opts);

/* Queue request *req (HOST struct; its device buffers and its host positions
 * must stay valid, and unchanged, until poll returns its ticket).  Outputs and
 * req->stats are written by the server; stats.status is the request's code as
 * clsimg_solve would return it.  *ticket > 0 identifies it.  Does no GPU work. */
int clsimg_server_submit(clsimg_server* srv, clsimg_request* req, int64_t* ticket);

/* Admit, run one round of steps, retire; with wait != 0 repeat until at least
 * one request is finished or the server holds no work.  Writes up to cap
 * finished tickets (their outputs complete on the device) to tickets[] and the
 * count to *n_done.  Returns CLSIMG_OK or an error of the server itself. */
int clsimg_server_poll(clsimg_server* srv, int32_t wait, int64_t* tickets, int32_t cap, int32_t* n_done);

/* Counters of the server (host struct). */
int clsimg_server_query(clsimg_server* srv, clsimg_server_info* info);

/* Stop the workers (after their current solves), wait for the streams and free
 * everything; requests not yet returned are abandoned. */
int clsimg_server_destroy(clsimg_server* srv);

/* Static description of a status code. */
const char* clsimg_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* CLSIMG_H */
