// C ABI of the clsimg library: context, workspace, steering tables and the
// host driver of the active-set solve (Table I of the paper) whose every
// arithmetic step runs in the kernels of ops.hip / solve.hip.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <limits>
#include <vector>

#include "../../include/clsimg.h"
#include "kernels.h"
#include "request.h"

using namespace clsimg;

namespace {

// refined multipliers: at most Q / 8 (64 .. this many) FP32 candidates per
// step (else the step's multipliers are all evaluated in FP32), and the |W|
// partial count
constexpr int kCandCap = 16384;
constexpr int kCandAbsParts = 256;

struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

struct TableKey {
  int P = -1;
  double lambda = 0.0;
  std::vector<double> pos;
  clsimg_grid grid{};
};

}  // namespace

struct clsimg_ctx {
  int device = 0;
  size_t budget = 0;  // 0 = unlimited
  size_t used = 0;
  // steering tables of the last (array, grid)
  TableKey key;
  bool tables_valid = false;
  DevBuf El, Em, pos_d;
  double* h_stage = nullptr;  // pinned staging for the antenna positions
  size_t h_stage_bytes = 0;
  hipEvent_t stage_done = nullptr;
  // workspace
  DevBuf frag_r, frag_u, frag_b, part, beta_part, alpha_part, keys;
  DevBuf B0, Bb, u, E, Rinv, W, Li;
  DevBuf Flist, Ulist, v, w, x, eps, mf, gamma;
  DevBuf lsqr, dec, status;
  DevBuf lsqr2, done, x1, w1, vraw, bpart0, bpart1, xf, bar;  // fused LSQR step
  DevBuf ostate;                                                // device-resident outer loop
  DevBuf pw_h, pw_rs, pw_g, pw_eps, pw_dinv, pw_Lw, pw_B0w;      // PWLS inputs
  DevBuf batch, batch_params, batch_rinv;                       // batched solve workspace
  // autotuned 16-pixel tiles per workgroup of the GEMM-shaped beamformers, by
  // precision (FP32, FP16, BF16) and row tiles per wave; 0: the default
  int tuned_nt[3][16] = {};
  char* h_batch = nullptr;                                      // pinned staging of the batch
  size_t h_batch_bytes = 0;
  SolveDecision* h_dec = nullptr;
  OuterState* h_outer = nullptr;
  LsqrState* h_lsqr = nullptr;
  int* h_status = nullptr;
  double* h_norms = nullptr;
  bool trace = false;  // CLSIMG_TRACE=1: one line per active-set step on stderr
  bool coop = false;   // cooperative launches available (multi-workgroup LSQR kernel)
  int lsqr_path = 0;   // CLSIMG_LSQR_PATH: 0 auto, 1 one workgroup, 2 cooperative, 3 two kernels/step
  bool old_beam = false;   // CLSIMG_LDS_BEAM=1: LDS-staged beamformer for the gradient
  bool beam_prep = false;  // CLSIMG_BEAM_PREP=1: beamformer fragments from a separate pass
  bool host_loop = false;  // CLSIMG_HOST_LOOP=1: active-set loop driven from the host
  int prec = CLSIMG_FP32;  // arithmetic of the full-grid beamforming products of the current call
  // K covariance blocks: per-block tables and vectors; tables_of() reads the
  // override while a block's operators run
  DevBuf mb_tab, mb_B0, mb_Bb, mb_u, mb_E, mb_frag, mb_acc, mb_acc2, mb_gpart;
  const float2* tab_El = nullptr;
  const float2* tab_Em = nullptr;
  double* h_mnorm = nullptr;  // pinned: the blocks' norm partials
  size_t h_mnorm_n = 0;
  DevBuf frag_h, hscale;   // half-precision fragments and their scale
  DevBuf mx_abs, mx_lam, mx_cand, mx_count;  // refined multipliers: |W| partials, lam~, candidates
  int outer_max_f = 1 << 30;  // CLSIMG_OUTER_MAXF: hand over to the host loop beyond this |F|
  void* scratch = nullptr;    // this device's copy of the static workspace (allocation-free calls)
  // device time of the host-driven loop's multiplier kernel (clsimg_kernel_timing)
  bool time_mult = false;
  hipEvent_t tm_ev[2] = {nullptr, nullptr};
  double tm_ms = 0.0;
  int tm_n = 0;
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// CLSIMG_VERBOSE=1: a failing HIP call names itself on stderr
int hip_failed(hipError_t e, int line) {
  static const bool verbose = [] {
    const char* v = getenv("CLSIMG_VERBOSE");
    return v && v[0] == '1';
  }();
  if (verbose) fprintf(stderr, "clsimg: %s (api.hip line %d)\n", hipGetErrorString(e), line);
  return CLSIMG_EHIP;
}

#define HIP_TRY(expr)                                    \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_failed(e_, __LINE__); \
  } while (0)

#define ST_TRY(expr)                  \
  do {                                \
    int s_ = (expr);                  \
    if (s_ != CLSIMG_OK) return s_;   \
  } while (0)

int ensure(clsimg_ctx* c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  if (b.bytes >= bytes) return CLSIMG_OK;
  if (c->budget && c->used - b.bytes + bytes > c->budget) return CLSIMG_ENOMEM;
  if (b.ptr) {
    (void)hipFree(b.ptr);
    c->used -= b.bytes;
    b.ptr = nullptr;
    b.bytes = 0;
  }
  if (hipMalloc(&b.ptr, bytes) != hipSuccess) return CLSIMG_ENOMEM;
  b.bytes = bytes;
  c->used += bytes;
  return CLSIMG_OK;
}

template <class T>
T* P_(DevBuf& b) {
  return reinterpret_cast<T*>(b.ptr);
}

int check_geometry(const clsimg_array* a, const clsimg_grid* g) {
  if (!a || !g || !a->pos_xy) return CLSIMG_EINVAL;
  if (a->P < 1 || a->P > CLSIMG_MAX_P) return CLSIMG_EINVAL;
  if (!(a->lambda > 0.0) || !isfinite(a->lambda)) return CLSIMG_EINVAL;
  if (g->nl < 1 || g->nm < 1) return CLSIMG_EINVAL;
  if ((int64_t)g->nl * g->nm > CLSIMG_MAX_Q) return CLSIMG_EINVAL;
  if (!isfinite(g->l0) || !isfinite(g->dl) || !isfinite(g->m0) || !isfinite(g->dm))
    return CLSIMG_EINVAL;
  for (int i = 0; i < 2 * a->P; ++i)
    if (!isfinite(a->pos_xy[i])) return CLSIMG_EINVAL;
  return CLSIMG_OK;
}

// Steering tables of (array, grid), rebuilt on the device only when either
// changes: positions go up through a pinned buffer, the FP64 phases and their
// complex64 rounding are computed by tables_kernel.
int ensure_tables(clsimg_ctx* c, const clsimg_array* a, const clsimg_grid* g, hipStream_t st) {
  const int P = a->P, Pp = pad_p(P);
  if (c->tables_valid && c->key.P == P && c->key.lambda == a->lambda &&
      memcmp(&c->key.grid, g, sizeof(*g)) == 0 &&
      memcmp(c->key.pos.data(), a->pos_xy, sizeof(double) * 2 * P) == 0)
    return CLSIMG_OK;
  ST_TRY(ensure(c, c->El, (size_t)Pp * g->nl * sizeof(float2)));
  ST_TRY(ensure(c, c->Em, (size_t)Pp * g->nm * sizeof(float2)));
  ST_TRY(ensure(c, c->pos_d, (size_t)2 * CLSIMG_MAX_P * sizeof(double)));
  if (!c->h_stage) {
    HIP_TRY(hipHostMalloc((void**)&c->h_stage, 2 * CLSIMG_MAX_P * sizeof(double), hipHostMallocDefault));
  } else {
    HIP_TRY(hipEventSynchronize(c->stage_done));  // the previous upload has left the buffer
  }
  memcpy(c->h_stage, a->pos_xy, sizeof(double) * 2 * P);
  HIP_TRY(hipMemcpyAsync(c->pos_d.ptr, c->h_stage, sizeof(double) * 2 * P, hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(c->stage_done, st));
  HIP_TRY(launch_tables(P_<const double>(c->pos_d), P, a->lambda, g->nl, g->nm, g->l0, g->dl, g->m0,
                        g->dm, P_<float2>(c->El), P_<float2>(c->Em), st));
  c->key.P = P;
  c->key.lambda = a->lambda;
  c->key.grid = *g;
  c->key.pos.assign(a->pos_xy, a->pos_xy + 2 * P);
  c->tables_valid = true;
  return CLSIMG_OK;
}

Tables tables_of(clsimg_ctx* c, const clsimg_grid* g, int P) {
  Tables t;
  t.El = c->tab_El ? c->tab_El : P_<const float2>(c->El);
  t.Em = c->tab_Em ? c->tab_Em : P_<const float2>(c->Em);
  t.nl = g->nl;
  t.nm = g->nm;
  t.Pp = pad_p(P);
  t.Q = g->nl * g->nm;
  return t;
}

AdjParams adj_params(clsimg_ctx* c, const clsimg_grid* g, int P, const float* frag, const int* idx,
                     int n, const int* stop, const float2* U = nullptr) {
  AdjParams pr;
  pr.frag = frag;
  pr.U = U;
  pr.xf = nullptr;
  pr.P = P;
  pr.MT = pad_p(P) / 8;
  pr.KS = pad_p(P) / 2;
  pr.tab = tables_of(c, g, P);
  pr.idx = idx;
  pr.n = n;
  pr.stop_flag = stop;
  return pr;
}

// partials of the correlation at its largest chunk count
size_t part_floats_max(int P) { return (size_t)forward_chunks_max(P) * forward_part_floats(P); }

int ntiles_adj(int P, int n) {
  const int T = adjoint_tile_width(pad_p(P) / 8);
  return (n + T - 1) / T;
}

// Common workspace for every operation on a problem of size (P, Q).
int ensure_workspace(clsimg_ctx* c, int P, int Q) {
  const int Pp = pad_p(P);
  const size_t fr = (size_t)4 * Pp * Pp * sizeof(float);
  const size_t cx = (size_t)P * P * sizeof(float2);
  ST_TRY(ensure(c, c->frag_r, fr));
  ST_TRY(ensure(c, c->frag_u, fr));
  ST_TRY(ensure(c, c->part, part_floats_max(P) * sizeof(float)));
  ST_TRY(ensure(c, c->beta_part, (size_t)reduce_blocks(P) * sizeof(double)));
  ST_TRY(ensure(c, c->alpha_part, (size_t)(ntiles_adj(P, Q) + 1) * sizeof(double)));
  ST_TRY(ensure(c, c->keys,
                (size_t)(std::max(ntiles_adj(P, Q), std::max(beam_grid(Q), beam_big_grid(P, Q, 2))) + 1) *
                    sizeof(uint64_t)));
  const size_t fb = beam_fits(P) ? (size_t)2 * (Pp / 8) * (Pp / 8 + 1) * 64
                                 : (beam_big_fits(P) ? beam_big_frag_floats(P) : 64);
  ST_TRY(ensure(c, c->frag_b, fb * sizeof(float)));
  ST_TRY(ensure(c, c->B0, cx));
  ST_TRY(ensure(c, c->Bb, cx));
  ST_TRY(ensure(c, c->u, cx));
  ST_TRY(ensure(c, c->E, cx));
  ST_TRY(ensure(c, c->Rinv, cx));
  ST_TRY(ensure(c, c->W, (size_t)2 * P * P * sizeof(double2)));  // L and its transpose (Cholesky beyond 64)
  ST_TRY(ensure(c, c->Li, (size_t)P * P * sizeof(double2)));
  ST_TRY(ensure(c, c->lsqr, sizeof(LsqrState)));
  ST_TRY(ensure(c, c->dec, sizeof(SolveDecision)));
  ST_TRY(ensure(c, c->status, 4 * sizeof(int)));
  return CLSIMG_OK;
}

// Psi_S v as the complex P x P matrix out = cK * K + cB * B (see RedParams).
int correlate(clsimg_ctx* c, const clsimg_grid* g, int P, const int* idx, const float* vals,
              int gather, int n, float2* out, const float2* B, float cK, float cB,
              const LsqrState* lsqr, float* frag, double* norm_part, const int* stop,
              hipStream_t st) {
  int chw = 16, nchunks = 0;
  forward_plan(P, n, &chw, &nchunks);
  const int MT = pad_p(P) / 8;
  if ((size_t)nchunks * forward_part_floats(P) > c->part.bytes / sizeof(float)) return CLSIMG_EINVAL;
  if (n > 0) {
    FwdParams f;
    f.tab = tables_of(c, g, P);
    f.MT = MT;
    f.idx = idx;
    f.vals = vals;
    f.gather = gather;
    f.n = n;
    f.chw = chw;
    f.part = P_<float>(c->part);
    f.stop_flag = stop;
    HIP_TRY(launch_forward(f, st));
  }
  RedParams r;
  r.part = P_<const float>(c->part);
  r.nchunks = n > 0 ? nchunks : 0;
  r.MT = MT;
  r.P = P;
  r.out = out;
  r.B = B;
  r.cK = cK;
  r.cB = cB;
  r.lsqr = lsqr;
  r.frag = frag;
  r.norm_part = norm_part;
  r.stop_flag = stop;
  HIP_TRY(launch_reduce(r, st));
  return CLSIMG_OK;
}

// correlate() over K covariance blocks in one forward and one reduction
// launch: block k uses the tables at tables_of() + k * tab_stride (float2) and
// reads / writes out, B, frag and norm_part at k times their strides.
int correlate_blocks(clsimg_ctx* c, const clsimg_grid* g, int P, int K, size_t tab_stride, const int* idx,
                     const float* vals, int gather, int n, float2* out, size_t out_stride, const float2* B,
                     size_t B_stride, float cK, float cB, const LsqrState* lsqr, float* frag, size_t frag_stride,
                     double* norm_part, size_t norm_stride, const int* stop, hipStream_t st) {
  int chw = 16, nchunks = 0;
  forward_plan(P, n, &chw, &nchunks);
  const int MT = pad_p(P) / 8;
  const size_t pstride = part_floats_max(P);
  if ((size_t)nchunks * forward_part_floats(P) > pstride || (size_t)K * pstride > c->part.bytes / sizeof(float))
    return CLSIMG_EINVAL;
  if (n > 0) {
    FwdParams f;
    f.tab = tables_of(c, g, P);
    f.MT = MT;
    f.idx = idx;
    f.vals = vals;
    f.gather = gather;
    f.n = n;
    f.chw = chw;
    f.part = P_<float>(c->part);
    f.stop_flag = stop;
    f.nblk = K;
    f.tab_stride = tab_stride;
    f.part_stride = pstride;
    HIP_TRY(launch_forward(f, st));
  }
  RedParams r;
  r.part = P_<const float>(c->part);
  r.nchunks = n > 0 ? nchunks : 0;
  r.MT = MT;
  r.P = P;
  r.out = out;
  r.B = B;
  r.cK = cK;
  r.cB = cB;
  r.lsqr = lsqr;
  r.frag = frag;
  r.norm_part = norm_part;
  r.stop_flag = stop;
  r.nblk = K;
  r.part_stride = pstride;
  r.out_stride = out_stride;
  r.B_stride = B_stride;
  r.frag_stride = frag_stride;
  r.norm_stride = norm_stride;
  HIP_TRY(launch_reduce(r, st));
  return CLSIMG_OK;
}

bool beam_any(int P) { return beam_fits(P) || beam_big_fits(P); }

// tiles per workgroup of the GEMM-shaped beamformer at the context's precision
int big_tiles(const clsimg_ctx* c, int P) {
  const int rpw = (pad_p(P) / 8 + 3) / 4;
  const int pr = c->prec == CLSIMG_FP16 ? 1 : (c->prec == CLSIMG_BF16 ? 2 : 0);
  return rpw < 16 ? c->tuned_nt[pr][rpw] : 0;
}

// Full-grid beamformer: for P <= 48 the block-triangular fragments of U stay
// in registers for the whole pass; for larger arrays (up to 288) the
// fragments are prepared once and streamed by the GEMM-shaped kernel.
enum BeamKind { BEAM_MF, BEAM_MVDR, BEAM_STORE };
int beam_full(clsimg_ctx* c, const clsimg_grid* g, int P, const float2* U, BeamKind kind, float* out,
              float* eps, float eps_scale, double C, double kb, float scale, hipStream_t st, Stamps ts = {}) {
  const Tables tab = tables_of(c, g, P);
  const Stamps first{ts.start, nullptr}, last{nullptr, ts.stop};  // a preparation pass, then the beamformer
  if (c->prec != CLSIMG_FP32) {  // split half precision, GEMM-shaped kernel for every P
    const bool bf = c->prec == CLSIMG_BF16;
    ST_TRY(ensure(c, c->frag_h, beam_h16_frag_bytes(P)));
    ST_TRY(ensure(c, c->hscale, sizeof(float)));
    HIP_TRY(launch_beam_prep_h16(U, P, bf, c->frag_h.ptr, P_<float>(c->hscale), st, first));
    const int k = kind == BEAM_MF ? 0 : (kind == BEAM_MVDR ? 1 : 2);
    HIP_TRY(launch_beam_h16(k, bf, c->frag_h.ptr, P_<const float>(c->hscale), tab, nullptr, out, eps, eps_scale, C,
                            kb, scale, nullptr, nullptr, st, last, big_tiles(c, P)));
    return CLSIMG_OK;
  }
  if (!beam_fits(P)) {  // larger arrays: fragments of the whole Ut, GEMM-shaped kernel
    HIP_TRY(launch_beam_prep_full(U, P, P_<float>(c->frag_b), st, first));
    const int k = kind == BEAM_MF ? 0 : (kind == BEAM_MVDR ? 1 : 2);
    HIP_TRY(launch_beam_big(k, P_<const float>(c->frag_b), tab, nullptr, out, eps, eps_scale, C, kb, scale,
                            nullptr, nullptr, st, last, big_tiles(c, P)));
    return CLSIMG_OK;
  }
  // fragments built inside the kernel, or prepared by a separate pass
  const float* fb = c->beam_prep ? P_<float>(c->frag_b) : nullptr;
  const float2* Uk = c->beam_prep ? nullptr : U;
  if (c->beam_prep) {
    HIP_TRY(launch_beam_prep(U, P, P_<float>(c->frag_b), st, first));
    ts = last;
  }
  switch (kind) {
    case BEAM_MF: HIP_TRY(launch_beam_mf(fb, Uk, P, tab, out, eps, eps_scale, st, ts)); break;
    case BEAM_MVDR: HIP_TRY(launch_beam_mvdr(fb, Uk, P, tab, out, C, kb, st)); break;
    default: HIP_TRY(launch_beam_store(fb, Uk, P, tab, out, scale, st)); break;
  }
  return CLSIMG_OK;
}

int read_back(clsimg_ctx* c, void* host, const void* dev, size_t bytes, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CLSIMG_OK;
}

double sum_host(const double* p, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += p[i];
  return s;
}

// MVDR / MF / NONE upper bound into `gamma`; MF image into `mf` if given.
int compute_bound(clsimg_ctx* c, const clsimg_c32* R, const clsimg_array* a, const clsimg_grid* g,
                  const clsimg_opts* o, float* gamma, hipStream_t st, const float2* rinv = nullptr) {
  const int P = a->P, Q = g->nl * g->nm;
  const float2* Rf = reinterpret_cast<const float2*>(R);
  if (o->bound == CLSIMG_BOUND_NONE) {
    HIP_TRY(launch_fill(gamma, std::numeric_limits<float>::infinity(), Q, st));
    return CLSIMG_OK;
  }
  if (o->bound == CLSIMG_BOUND_MF) {
    const double scale = 1.0 + (o->kappa_b != 0.0 ? o->kappa_b / sqrt((double)o->nsamples) : 0.0);
    if (beam_any(P)) return beam_full(c, g, P, Rf, BEAM_STORE, gamma, nullptr, 0.f, 0, 0, (float)scale, st);
    HIP_TRY(launch_adjoint_store(adj_params(c, g, P, nullptr, nullptr, Q, nullptr, Rf), gamma,
                                 (float)scale, st));
    return CLSIMG_OK;
  }
  if (!rinv) {  // else factored and checked beforehand (batched factorisation)
    HIP_TRY(launch_chol_inverse(Rf, P, P_<double2>(c->W), P_<double2>(c->Li), P_<float2>(c->Rinv),
                                P_<int>(c->status), st));
    ST_TRY(read_back(c, c->h_status, c->status.ptr, sizeof(int), st));
    if (*c->h_status != 0) return CLSIMG_ENOTPD;
    rinv = P_<const float2>(c->Rinv);
  }
  const double kb = o->kappa_b != 0.0 ? o->kappa_b / sqrt((double)(o->nsamples - P - 1)) : 0.0;
  if (beam_any(P)) return beam_full(c, g, P, rinv, BEAM_MVDR, gamma, nullptr, 0.f, o->C, kb, 1.f, st);
  HIP_TRY(launch_adjoint_mvdr(adj_params(c, g, P, nullptr, nullptr, Q, nullptr, rinv), gamma, o->C, kb, st));
  return CLSIMG_OK;
}

// Dense-count flops: a correlation over n pixels costs 8 P^2 n, a beamforming
// over n pixels 8 P^2 n + 8 P n (the complex GEMM and the column dot).
double corr_flops(int P, int n) { return 8.0 * P * P * n; }
double beam_flops(int P, int n) { return 8.0 * P * P * n + 8.0 * P * n; }

int check_opts(const clsimg_opts* o, int P) {
  if (!o) return CLSIMG_EINVAL;
  if (o->bound < CLSIMG_BOUND_MVDR || o->bound > CLSIMG_BOUND_NONE) return CLSIMG_EINVAL;
  if (o->precision != CLSIMG_FP32 && o->precision != CLSIMG_FP16 && o->precision != CLSIMG_BF16)
    return CLSIMG_EINVAL;
  if (o->cost != CLSIMG_COST_LS && o->cost != CLSIMG_COST_PWLS) return CLSIMG_EINVAL;
  if (o->cost == CLSIMG_COST_PWLS && !(o->C > 0.0)) return CLSIMG_EINVAL;
  if (o->bound == CLSIMG_BOUND_MVDR && !(o->C > 0.0)) return CLSIMG_EINVAL;
  if (o->kappa_b != 0.0) {
    if (o->bound == CLSIMG_BOUND_MVDR && o->nsamples <= P + 1) return CLSIMG_EINVAL;
    if (o->bound == CLSIMG_BOUND_MF && o->nsamples <= 0) return CLSIMG_EINVAL;
  }
  if (!(o->kappa_d >= 0.0) || !(o->kappa_b >= 0.0)) return CLSIMG_EINVAL;
  if (!(o->atol >= 0.0) || !(o->btol >= 0.0) || !(o->conlim > 0.0)) return CLSIMG_EINVAL;
  return CLSIMG_OK;
}

}  // namespace

namespace clsimg {

bool request_on_device(int P) { return beam_fits(P) && outer_fits(P); }

ReqLayout request_layout(int P, int nl, int nm, bool pwls, int nkeys) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const int Pp = pad_p(P);
  const size_t Q = (size_t)nl * nm;
  ReqLayout L;
  L.nkeys = nkeys;
  L.El = 0;
  L.Em = L.El + al((size_t)Pp * nl * sizeof(float2));
  L.B0 = L.Em + al((size_t)Pp * nm * sizeof(float2));
  L.Bb = L.B0 + al((size_t)P * P * sizeof(float2));
  L.E = L.Bb + al((size_t)P * P * sizeof(float2));
  L.eps = L.E + al((size_t)P * P * sizeof(float2));
  L.gam = L.eps + al(Q * sizeof(float));
  L.mf = L.gam + al(Q * sizeof(float));
  L.F = L.mf + al(Q * sizeof(float));
  L.U = L.F + al(Q * sizeof(int));
  L.st = L.U + al(2 * Q * sizeof(int));
  L.keys = L.st + al(sizeof(OuterState));
  L.rs = L.keys + al((size_t)nkeys * sizeof(uint64_t));
  L.gpw = L.rs + (pwls ? al(Q * sizeof(float)) : 0);
  L.dinv = L.gpw + (pwls ? al(Q * sizeof(float)) : 0);
  L.Lw = L.dinv + (pwls ? al(Q * sizeof(float)) : 0);
  L.bytes = L.Lw + (pwls ? al((size_t)P * P * sizeof(float2)) : 0);
  return L;
}

int request_setup(clsimg_ctx* c, clsimg_request& q, const clsimg_opts* o, char* slice, const ReqLayout& L,
                  OuterParams& op, BeamLamItem& it, hipStream_t st, const float2* rinv, const SetupItems* defer) {
  memset(&q.stats, 0, sizeof(clsimg_stats));
  c->prec = o->precision;
  const int P = q.array.P, Pp = pad_p(P);
  const int Q = q.grid.nl * q.grid.nm;
  const bool pwls = o->cost == CLSIMG_COST_PWLS;
  ST_TRY(ensure_workspace(c, P, Q));
  ST_TRY(ensure(c, c->eps, (size_t)Q * sizeof(float)));
  if (pwls) ST_TRY(ensure(c, c->pw_h, (size_t)Q * sizeof(float)));
  const float2* Rf = reinterpret_cast<const float2*>(q.R);
  // the steering tables: built in the context, then kept in the slice
  const float2* El;
  const float2* Em;
  if (defer && !defer->shared_tables) {  // built into the slice by the batched tables launch
    float2* sl = reinterpret_cast<float2*>(slice + L.El);
    float2* sm = reinterpret_cast<float2*>(slice + L.Em);
    memcpy(defer->pos_host, q.array.pos_xy, sizeof(double) * 2 * P);
    const clsimg_grid& g = q.grid;
    *defer->table = TableItem{defer->pos_dev, q.array.lambda, g.l0, g.dl, g.m0, g.dm, P, g.nl, g.nm, sl, sm};
    El = sl;
    Em = sm;
  } else {
    ST_TRY(ensure_tables(c, &q.array, &q.grid, st));
    El = P_<const float2>(c->El);
    Em = P_<const float2>(c->Em);
    if (!defer) {
      float2* sl = reinterpret_cast<float2*>(slice + L.El);
      float2* sm = reinterpret_cast<float2*>(slice + L.Em);
      HIP_TRY(hipMemcpyAsync(sl, El, (size_t)Pp * q.grid.nl * sizeof(float2), hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(sm, Em, (size_t)Pp * q.grid.nm * sizeof(float2), hipMemcpyDeviceToDevice, st));
      El = sl;
      Em = sm;
    }
  }
  Tables tab;
  tab.El = El;
  tab.Em = Em;
  tab.nl = q.grid.nl;
  tab.nm = q.grid.nm;
  tab.Pp = Pp;
  tab.Q = Q;
  const float eps_scale = o->kappa_d != 0.0 ? (float)(o->kappa_d / sqrt((double)o->nsamples)) : 0.f;
  float* eps = reinterpret_cast<float*>(slice + L.eps);
  float* mf = q.mf ? q.mf : reinterpret_cast<float*>(slice + L.mf);
  float* gamma = q.gamma ? q.gamma : reinterpret_cast<float*>(slice + L.gam);
  float2* B0 = reinterpret_cast<float2*>(slice + L.B0);
  OuterState* ost = reinterpret_cast<OuterState*>(slice + L.st);
  const int nblk = beam_grid_batched(Q, L.tiles);
  if (nblk > L.nkeys) return CLSIMG_EINVAL;
  if (defer) {
    if (pwls || !rinv || o->bound != CLSIMG_BOUND_MVDR || c->prec != CLSIMG_FP32 || !beam_fits(P) || c->beam_prep)
      return CLSIMG_EINVAL;
    const double kb = o->kappa_b != 0.0 ? o->kappa_b / sqrt((double)(o->nsamples - P - 1)) : 0.0;
    *defer->beam = BeamSetItem{Rf, rinv, tab, mf, eps, gamma, eps_scale, o->C, kb, P, nblk};
    *defer->init = ReqInitItem{Rf, q.noise_diag, B0, q.sigma, q.state, ost, P, Q};
  } else {
    ST_TRY(beam_full(c, &q.grid, P, Rf, BEAM_MF, mf, eps, eps_scale, 0, 0, 1.f, st));
    ST_TRY(compute_bound(c, q.R, &q.array, &q.grid, o, gamma, st, rinv));
  }
  const float* op_gamma = gamma;
  const float* rowscale = nullptr;
  const float2* Lw = nullptr;
  const float* dinv = nullptr;
  if (!pwls) {
    if (!defer) HIP_TRY(launch_sub_diag(Rf, q.noise_diag, P, B0, st));
  } else {
    if (o->bound != CLSIMG_BOUND_MVDR) {
      HIP_TRY(launch_chol_inverse(Rf, P, P_<double2>(c->W), P_<double2>(c->Li), P_<float2>(c->Rinv),
                                  P_<int>(c->status), st));
      ST_TRY(read_back(c, c->h_status, c->status.ptr, sizeof(int), st));
      if (*c->h_status != 0) return CLSIMG_ENOTPD;
    }
    float* h = P_<float>(c->pw_h);
    ST_TRY(beam_full(c, &q.grid, P, P_<const float2>(c->Rinv), BEAM_STORE, h, nullptr, 0.f, 0, 0, 1.f, st));
    const double kd = o->kappa_d != 0.0 ? o->kappa_d / sqrt((double)(o->nsamples - P - 1)) : 0.0;
    float* rs = reinterpret_cast<float*>(slice + L.rs);
    float* gpw = reinterpret_cast<float*>(slice + L.gpw);
    float* dv = reinterpret_cast<float*>(slice + L.dinv);
    float2* lw = reinterpret_cast<float2*>(slice + L.Lw);
    HIP_TRY(launch_pwls_setup(h, gamma, o->C, kd, Q, rs, gpw, eps, dv, st));
    HIP_TRY(launch_sub_diag(Rf, q.noise_diag, P, P_<float2>(c->B0), st));
    HIP_TRY(launch_pwls_whiten(P_<const double2>(c->Li), P_<const float2>(c->B0), P, lw, B0, st));
    op_gamma = gpw;
    rowscale = rs;
    Lw = lw;
    dinv = dv;
  }
  if (!defer) {
    HIP_TRY(launch_init_state(nullptr, nullptr, q.sigma, q.state, Q, st));
    HIP_TRY(launch_outer_init(ost, nullptr, st));
  }
  op.st = ost;
  op.Flist = reinterpret_cast<int*>(slice + L.F);
  op.Ulist = reinterpret_cast<int*>(slice + L.U);
  op.sigma = q.sigma;
  op.gamma = op_gamma;
  op.eps = eps;
  op.state = q.state;
  op.B0 = B0;
  op.Bb = reinterpret_cast<float2*>(slice + L.Bb);
  op.E = reinterpret_cast<float2*>(slice + L.E);
  op.keys = reinterpret_cast<const uint64_t*>(slice + L.keys);
  op.nkeys = nblk;
  op.tab = tab;
  op.P = P;
  op.Q = Q;
  op.atol = o->atol;
  op.btol = o->btol;
  op.conlim = o->conlim;
  op.itnlim = o->itnlim;
  op.max_outer = o->max_outer < 0 ? 4 * Q : o->max_outer;
  op.max_f = c->outer_max_f;
  op.Lw = Lw;
  op.rowscale = rowscale;
  it.U = op.E;
  it.tab = tab;
  it.skip = &ost->lam_skip;
  it.state = q.state;
  it.part = reinterpret_cast<uint64_t*>(slice + L.keys);
  it.scale = dinv;
  it.P = P;
  it.nblk = nblk;
  return CLSIMG_OK;
}

int request_finish(clsimg_request& q, const clsimg_opts* o, char* slice, const ReqLayout& L, const OuterState& S,
                   hipStream_t st) {
  const int P = q.array.P;
  const int Q = q.grid.nl * q.grid.nm;
  int status = S.status == kStatusMaxOuter ? CLSIMG_WMAXOUTER : (S.status == kStatusCycle ? CLSIMG_WCYCLE : CLSIMG_OK);
  if (status == CLSIMG_OK && S.itnlim_hits) status = CLSIMG_WITNLIM;
  if (S.fallback) status = CLSIMG_ENOTSUP;
  if (o->cost == CLSIMG_COST_PWLS && !S.fallback)
    HIP_TRY(launch_pwls_scale(q.sigma, reinterpret_cast<const float*>(slice + L.dinv), Q, false, st));
  clsimg_stats& t = q.stats;
  t.status = status;
  t.outer_iters = S.outer;
  t.adds = S.adds;
  t.drops = S.drops;
  t.lsqr_iters_total = S.lsqr_total;
  t.lsqr_itnlim_hits = S.itnlim_hits;
  t.nF = S.nF;
  t.nU = S.nU;
  t.rel_residual = S.b0n2 > 0.0 ? sqrt(S.res2 / S.b0n2) : 0.0;
  t.objective = 0.5 * S.res2;
  t.min_margin_lambda = S.margin_lambda;
  t.min_margin_z = S.margin_z;
  t.psi_flops = S.psi_flops + beam_flops(P, Q) + (o->bound != CLSIMG_BOUND_NONE ? beam_flops(P, Q) : 0.0);
  return status;
}

}  // namespace clsimg

namespace {

// Static workspace of the allocation-free dirty image: every GPU the library
// runs on holds one copy until the process ends.  Host code never uses the
// array's name as an address: clsimg_create resolves this device's copy with
// hipGetSymbolAddress and keeps it in the context.
constexpr size_t kNoAllocBytes = (size_t)8 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

}  // namespace

extern "C" {

void clsimg_default_opts(clsimg_opts* o) {
  if (!o) return;
  o->bound = CLSIMG_BOUND_MVDR;
  o->C = 1.0;
  o->kappa_b = 0.0;
  o->kappa_d = 6.0;
  o->nsamples = 0;
  o->atol = 1e-6;
  o->btol = 1e-6;
  o->conlim = 1e8;
  o->itnlim = -1;
  o->max_outer = -1;
  o->precision = CLSIMG_FP32;
  o->cost = CLSIMG_COST_LS;
}

int clsimg_create(clsimg_ctx** out, int32_t device, size_t budget) {
  if (!out) return CLSIMG_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return CLSIMG_EINVAL;
  DeviceGuard guard(device);
  clsimg_ctx* c = new (std::nothrow) clsimg_ctx();
  if (!c) return CLSIMG_ENOMEM;
  c->device = device;
  c->budget = budget;
  const char* tr = getenv("CLSIMG_TRACE");
  c->trace = tr && tr[0] == '1';
  int coop = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) == hipSuccess)
    c->coop = coop != 0;
  const char* lp = getenv("CLSIMG_LSQR_PATH");
  if (lp) c->lsqr_path = atoi(lp);
  const char* ob = getenv("CLSIMG_LDS_BEAM");
  c->old_beam = ob && ob[0] == '1';
  const char* bp = getenv("CLSIMG_BEAM_PREP");
  c->beam_prep = bp && bp[0] == '1';
  const char* hl = getenv("CLSIMG_HOST_LOOP");
  c->host_loop = hl && hl[0] == '1';
  const char* mf_ = getenv("CLSIMG_OUTER_MAXF");
  if (mf_) c->outer_max_f = atoi(mf_);
  void* hp = nullptr;
  // room for the norm partials of the largest array (reduce_blocks grows as P^2)
  const int nnorm = reduce_blocks(CLSIMG_MAX_P);
  const size_t hbytes =
      sizeof(SolveDecision) + sizeof(LsqrState) + 4 * sizeof(int) + nnorm * sizeof(double) + sizeof(OuterState);
  if (hipHostMalloc(&hp, hbytes, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming) != hipSuccess) {
    if (hp) (void)hipHostFree(hp);
    delete c;
    return CLSIMG_EHIP;
  }
  char* b = static_cast<char*>(hp);
  c->h_dec = reinterpret_cast<SolveDecision*>(b);
  c->h_lsqr = reinterpret_cast<LsqrState*>(b + sizeof(SolveDecision));
  c->h_status = reinterpret_cast<int*>(b + sizeof(SolveDecision) + sizeof(LsqrState));
  c->h_norms = reinterpret_cast<double*>(b + sizeof(SolveDecision) + sizeof(LsqrState) + 4 * sizeof(int));
  c->h_outer = reinterpret_cast<OuterState*>(b + sizeof(SolveDecision) + sizeof(LsqrState) + 4 * sizeof(int) +
                                             nnorm * sizeof(double));
  // this device's copy of the static workspace (the device is current here)
  void* sp = nullptr;
  if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) {
    (void)hipHostFree(hp);
    (void)hipEventDestroy(c->stage_done);
    delete c;
    return CLSIMG_EHIP;
  }
  c->scratch = sp;
  *out = c;
  return CLSIMG_OK;
}

int clsimg_destroy(clsimg_ctx* c) {
  if (!c) return CLSIMG_EINVAL;
  DeviceGuard guard(c->device);
  (void)hipDeviceSynchronize();
  DevBuf* bufs[] = {&c->El,   &c->Em,    &c->pos_d,    &c->frag_r, &c->frag_u, &c->frag_b, &c->ostate, &c->pw_h, &c->pw_rs, &c->pw_g, &c->pw_eps, &c->pw_dinv, &c->pw_Lw, &c->pw_B0w, &c->batch, &c->batch_params, &c->batch_rinv, &c->part,  &c->beta_part,
                    &c->alpha_part, &c->keys, &c->B0, &c->Bb,   &c->u,     &c->E,
                    &c->Rinv, &c->W,     &c->Li,     &c->Flist,  &c->Ulist, &c->v,
                    &c->w,    &c->x,     &c->eps,    &c->mf,     &c->gamma, &c->lsqr,
                    &c->dec,  &c->status, &c->lsqr2, &c->done, &c->x1, &c->w1, &c->vraw,
                    &c->bpart0, &c->bpart1, &c->xf, &c->bar, &c->frag_h, &c->hscale,
                    &c->mx_abs, &c->mx_lam, &c->mx_cand, &c->mx_count,
                    &c->mb_tab, &c->mb_B0, &c->mb_Bb, &c->mb_u, &c->mb_E, &c->mb_frag, &c->mb_acc, &c->mb_acc2,
                    &c->mb_gpart};
  for (DevBuf* d : bufs)
    if (d->ptr) (void)hipFree(d->ptr);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  if (c->h_dec) (void)hipHostFree(c->h_dec);
  if (c->h_batch) (void)hipHostFree(c->h_batch);
  if (c->h_mnorm) (void)hipHostFree(c->h_mnorm);
  if (c->stage_done) (void)hipEventDestroy(c->stage_done);
  for (hipEvent_t e : c->tm_ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
  return CLSIMG_OK;
}

const char* clsimg_strerror(int s) {
  switch (s) {
    case CLSIMG_OK: return "ok";
    case CLSIMG_WMAXOUTER: return "active-set iteration limit reached";
    case CLSIMG_WITNLIM: return "an LSQR subproblem reached its iteration limit";
    case CLSIMG_WCYCLE: return "released pixel blocked again at zero step (cycle)";
    case CLSIMG_EINVAL: return "invalid argument";
    case CLSIMG_ENOTPD: return "covariance is not positive definite or not finite";
    case CLSIMG_ENOMEM: return "workspace exceeds the HBM budget or allocation failed";
    case CLSIMG_EHIP: return "HIP runtime error";
    case CLSIMG_ENOTSUP: return "option not available for this problem size";
    default: return "unknown status";
  }
}

int clsimg_dirty_image(clsimg_ctx* c, const clsimg_c32* R, const clsimg_array* a,
                       const clsimg_grid* g, int32_t precision, float* mf, void* stream) {
  if (!c || !R || !mf) return CLSIMG_EINVAL;
  ST_TRY(check_geometry(a, g));
  if (precision != CLSIMG_FP32 && precision != CLSIMG_FP16 && precision != CLSIMG_BF16) return CLSIMG_EINVAL;
  c->prec = precision;
  DeviceGuard guard(c->device);
  hipStream_t st = (hipStream_t)stream;
  const int P = a->P, Q = g->nl * g->nm;
  ST_TRY(ensure_workspace(c, P, Q));
  ST_TRY(ensure_tables(c, a, g, st));
  const float2* Rf = reinterpret_cast<const float2*>(R);
  if (beam_any(P)) return beam_full(c, g, P, Rf, BEAM_MF, mf, nullptr, 0.f, 0, 0, 1.f, st);
  HIP_TRY(launch_adjoint_mf(adj_params(c, g, P, nullptr, nullptr, Q, nullptr, Rf), mf, nullptr, 0.f, st));
  return CLSIMG_OK;
}

int clsimg_set_beam_tiles(clsimg_ctx* c, int32_t P, int32_t precision, int32_t tiles) {
  if (!c || P < 1 || P > CLSIMG_MAX_P) return CLSIMG_EINVAL;
  if (precision != CLSIMG_FP32 && precision != CLSIMG_FP16 && precision != CLSIMG_BF16) return CLSIMG_EINVAL;
  if (tiles != 0 && !beam_tiles_offered(precision != CLSIMG_FP32, tiles, (pad_p(P) / 8 + 3) / 4)) return CLSIMG_EINVAL;
  const int pr = precision == CLSIMG_FP16 ? 1 : (precision == CLSIMG_BF16 ? 2 : 0);
  c->tuned_nt[pr][(pad_p(P) / 8 + 3) / 4] = tiles;
  return CLSIMG_OK;
}

int clsimg_kernel_timing(clsimg_ctx* c, int32_t enable, double* ms, int32_t* launches) {
  if (!c) return CLSIMG_EINVAL;
  if (ms) *ms = c->tm_ms;
  if (launches) *launches = c->tm_n;
  c->tm_ms = 0.0;
  c->tm_n = 0;
  if (enable && !c->tm_ev[0]) {
    DeviceGuard guard(c->device);
    for (hipEvent_t& e : c->tm_ev) HIP_TRY(hipEventCreate(&e));
  }
  c->time_mult = enable != 0;
  return CLSIMG_OK;
}

int clsimg_autotune(clsimg_ctx* c, const clsimg_array* a, const clsimg_grid* g, int32_t precision, int32_t* chosen,
                    float* us, void* stream) {
  if (!c) return CLSIMG_EINVAL;
  ST_TRY(check_geometry(a, g));
  if (precision != CLSIMG_FP32 && precision != CLSIMG_FP16 && precision != CLSIMG_BF16) return CLSIMG_EINVAL;
  const int P = a->P, Q = g->nl * g->nm;
  if (!beam_big_fits(P) || (precision == CLSIMG_FP32 && beam_fits(P))) return CLSIMG_ENOTSUP;
  c->prec = precision;
  DeviceGuard guard(c->device);
  hipStream_t st = (hipStream_t)stream;
  ST_TRY(ensure_workspace(c, P, Q));
  ST_TRY(ensure_tables(c, a, g, st));
  ST_TRY(ensure(c, c->mf, (size_t)Q * sizeof(float)));
  // a synthetic covariance (the identity): the kernels' time does not depend on the values
  std::vector<float2> eye((size_t)P * P, make_float2(0.f, 0.f));
  for (int p = 0; p < P; ++p) eye[(size_t)p * P + p] = make_float2(1.f, 0.f);
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipMemcpy(c->B0.ptr, eye.data(), eye.size() * sizeof(float2), hipMemcpyHostToDevice));
  const int pr = precision == CLSIMG_FP16 ? 1 : (precision == CLSIMG_BF16 ? 2 : 0);
  const int rpw = (pad_p(P) / 8 + 3) / 4;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return CLSIMG_EHIP;
  }
  int status = CLSIMG_OK, best = 0;
  float tbest = 0.f;
  const int reps = 5;
  for (int i = 0; i < 3 && status == CLSIMG_OK; ++i) {
    const int nt = kBigTileChoices[i];
    if (!beam_tiles_offered(precision != CLSIMG_FP32, nt, rpw)) {  // not built
      if (us) us[i] = -1.f;
      continue;
    }
    c->tuned_nt[pr][rpw] = nt;
    float ms = 0.f;
    for (int w = 0; w < 2 && status == CLSIMG_OK; ++w)
      status = beam_full(c, g, P, P_<const float2>(c->B0), BEAM_MF, P_<float>(c->mf), nullptr, 0.f, 0, 0, 1.f, st);
    if (status == CLSIMG_OK && hipEventRecord(e0, st) != hipSuccess) status = CLSIMG_EHIP;
    for (int r = 0; r < reps && status == CLSIMG_OK; ++r)
      status = beam_full(c, g, P, P_<const float2>(c->B0), BEAM_MF, P_<float>(c->mf), nullptr, 0.f, 0, 0, 1.f, st);
    if (status == CLSIMG_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      status = CLSIMG_EHIP;
    if (status != CLSIMG_OK) break;
    const float t = 1e3f * ms / reps;
    if (us) us[i] = t;
    if (best == 0 || t < tbest) {
      best = nt;
      tbest = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tuned_nt[pr][rpw] = status == CLSIMG_OK ? best : 0;
  if (chosen) *chosen = c->tuned_nt[pr][rpw];
  return status;
}

int clsimg_dirty_image_timed(clsimg_ctx* c, const clsimg_c32* R, const clsimg_array* a, const clsimg_grid* g,
                             int32_t precision, float* mf, void* start_event, void* stop_event, void* stream) {
  if (!c || !R || !mf || !start_event || !stop_event) return CLSIMG_EINVAL;
  ST_TRY(check_geometry(a, g));
  if (precision != CLSIMG_FP32 && precision != CLSIMG_FP16 && precision != CLSIMG_BF16) return CLSIMG_EINVAL;
  if (!beam_any(a->P)) return CLSIMG_ENOTSUP;
  c->prec = precision;
  DeviceGuard guard(c->device);
  hipStream_t st = (hipStream_t)stream;
  const int P = a->P, Q = g->nl * g->nm;
  ST_TRY(ensure_workspace(c, P, Q));
  ST_TRY(ensure_tables(c, a, g, st));
  const Stamps ts{(hipEvent_t)start_event, (hipEvent_t)stop_event};
  return beam_full(c, g, P, reinterpret_cast<const float2*>(R), BEAM_MF, mf, nullptr, 0.f, 0, 0, 1.f, st, ts);
}

int clsimg_dirty_image_noalloc(clsimg_ctx* c, const clsimg_c32* R, const clsimg_array* a, const clsimg_grid* g,
                               int32_t precision, float* mf, void* stream) {
  if (!c || !R || !mf || !c->scratch) return CLSIMG_EINVAL;
  ST_TRY(check_geometry(a, g));
  if (precision != CLSIMG_FP32 && precision != CLSIMG_FP16 && precision != CLSIMG_BF16) return CLSIMG_EINVAL;
  const int P = a->P, Pp = pad_p(P), Q = g->nl * g->nm;
  if (!beam_any(P)) return CLSIMG_ENOTSUP;
  // workspace layout: positions | El | Em | fragments | FP16 scale
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t o_pos = take((size_t)2 * P * sizeof(double));
  const size_t o_el = take((size_t)Pp * g->nl * sizeof(float2));
  const size_t o_em = take((size_t)Pp * g->nm * sizeof(float2));
  size_t fb = 0;
  if (precision != CLSIMG_FP32) fb = beam_h16_frag_bytes(P);
  else if (!beam_fits(P)) fb = beam_big_frag_floats(P) * sizeof(float);
  const size_t o_fr = take(fb), o_sc = take(sizeof(float));
  if (off > kNoAllocBytes) return CLSIMG_ENOMEM;
  c->prec = precision;
  DeviceGuard guard(c->device);
  hipStream_t st = (hipStream_t)stream;
  unsigned char* base = static_cast<unsigned char*>(c->scratch);
  double* pos = reinterpret_cast<double*>(base + o_pos);
  Tables tab;
  tab.El = reinterpret_cast<const float2*>(base + o_el);
  tab.Em = reinterpret_cast<const float2*>(base + o_em);
  tab.nl = g->nl;
  tab.nm = g->nm;
  tab.Pp = Pp;
  tab.Q = Q;
  HIP_TRY(hipMemcpyAsync(pos, a->pos_xy, (size_t)2 * P * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(launch_tables(pos, P, a->lambda, g->nl, g->nm, g->l0, g->dl, g->m0, g->dm,
                        reinterpret_cast<float2*>(base + o_el), reinterpret_cast<float2*>(base + o_em), st));
  const float2* Rf = reinterpret_cast<const float2*>(R);
  if (precision != CLSIMG_FP32) {
    const bool bf = precision == CLSIMG_BF16;
    float* sc = reinterpret_cast<float*>(base + o_sc);
    HIP_TRY(launch_beam_prep_h16(Rf, P, bf, base + o_fr, sc, st));
    HIP_TRY(launch_beam_h16(0, bf, base + o_fr, sc, tab, nullptr, mf, nullptr, 0.f, 0, 0, 1.f, nullptr, nullptr, st,
                            {}, big_tiles(c, P)));
  } else if (!beam_fits(P)) {
    float* fr = reinterpret_cast<float*>(base + o_fr);
    HIP_TRY(launch_beam_prep_full(Rf, P, fr, st));
    HIP_TRY(launch_beam_big(0, fr, tab, nullptr, mf, nullptr, 0.f, 0, 0, 1.f, nullptr, nullptr, st, {},
                            big_tiles(c, P)));
  } else {
    HIP_TRY(launch_beam_mf(nullptr, Rf, P, tab, mf, nullptr, 0.f, st));
  }
  return CLSIMG_OK;
}

int clsimg_mvdr_bound(clsimg_ctx* c, const clsimg_c32* R, const clsimg_array* a,
                      const clsimg_grid* g, const clsimg_opts* o, float* gamma, void* stream) {
  if (!c || !R || !gamma) return CLSIMG_EINVAL;
  ST_TRY(check_geometry(a, g));
  ST_TRY(check_opts(o, a->P));
  c->prec = o->precision;
  DeviceGuard guard(c->device);
  hipStream_t st = (hipStream_t)stream;
  ST_TRY(ensure_workspace(c, a->P, g->nl * g->nm));
  ST_TRY(ensure_tables(c, a, g, st));
  return compute_bound(c, R, a, g, o, gamma, st);
}

int clsimg_forward(clsimg_ctx* c, const clsimg_array* a, const clsimg_grid* g, const int32_t* idx,
                   const float* v, int32_t n, clsimg_c32* Y, void* stream) {
  if (!c || !Y || n < 0 || (n > 0 && !v)) return CLSIMG_EINVAL;
  ST_TRY(check_geometry(a, g));
  if (!idx && n > g->nl * g->nm) return CLSIMG_EINVAL;
  c->prec = CLSIMG_FP32;
  DeviceGuard guard(c->device);
  hipStream_t st = (hipStream_t)stream;
  ST_TRY(ensure_workspace(c, a->P, g->nl * g->nm));
  ST_TRY(ensure_tables(c, a, g, st));
  return correlate(c, g, a->P, idx, v, 0, n, reinterpret_cast<float2*>(Y), nullptr, 1.f, 0.f, nullptr,
                   nullptr, nullptr, nullptr, st);
}

int clsimg_adjoint(clsimg_ctx* c, const clsimg_array* a, const clsimg_grid* g, const clsimg_c32* U,
                   const int32_t* idx, int32_t n, float* out, void* stream) {
  if (!c || !U || n < 0 || (n > 0 && !out)) return CLSIMG_EINVAL;
  ST_TRY(check_geometry(a, g));
  if (!idx && n > g->nl * g->nm) return CLSIMG_EINVAL;
  DeviceGuard guard(c->device);
  hipStream_t st = (hipStream_t)stream;
  const int P = a->P;
  ST_TRY(ensure_workspace(c, P, std::max(n, g->nl * g->nm)));
  ST_TRY(ensure_tables(c, a, g, st));
  if (n == 0) return CLSIMG_OK;
  if (!idx && n == g->nl * g->nm && beam_any(P))
    return beam_full(c, g, P, reinterpret_cast<const float2*>(U), BEAM_STORE, out, nullptr, 0.f, 0, 0, 1.f,
                     st);
  HIP_TRY(launch_adjoint_store(
      adj_params(c, g, P, nullptr, idx, n, nullptr, reinterpret_cast<const float2*>(U)), out, 1.f, st));
  return CLSIMG_OK;
}

int clsimg_solve(clsimg_ctx* c, const clsimg_c32* R, const clsimg_array* a, const clsimg_grid* g,
                 const float* noise_diag, const clsimg_opts* o, const float* sigma0,
                 const uint8_t* state0, float* sigma, uint8_t* state, float* mf_out,
                 float* gamma_out, clsimg_stats* stats, void* stream) {
  if (stats) memset(stats, 0, sizeof(*stats));
  if (!c || !R || !sigma || !state || !stats) return CLSIMG_EINVAL;
  if ((sigma0 == nullptr) != (state0 == nullptr)) return CLSIMG_EINVAL;
  ST_TRY(check_geometry(a, g));
  ST_TRY(check_opts(o, a->P));
  if (o->nsamples <= 0 && o->kappa_d != 0.0) return CLSIMG_EINVAL;
  c->prec = o->precision;
  DeviceGuard guard(c->device);
  hipStream_t st = (hipStream_t)stream;
  const int P = a->P, Q = g->nl * g->nm;
  ST_TRY(ensure_workspace(c, P, Q));
  ST_TRY(ensure(c, c->Flist, (size_t)Q * sizeof(int)));
  ST_TRY(ensure(c, c->Ulist, (size_t)2 * Q * sizeof(int)));  // two buffers for the device loop
  ST_TRY(ensure(c, c->ostate, sizeof(OuterState)));
  ST_TRY(ensure(c, c->v, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->w, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->x, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->x1, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->w1, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->vraw, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->lsqr2, 3 * sizeof(LsqrState)));
  ST_TRY(ensure(c, c->done, sizeof(int)));
  ST_TRY(ensure(c, c->bar, 2 * sizeof(unsigned)));
  {
    const int nparts = std::max(std::max(reduce_blocks(P), lsqr_fwd_waves(P)), Q / 32 + 64);
    const size_t nb = (size_t)nparts * sizeof(double);
    ST_TRY(ensure(c, c->bpart0, nb));
    ST_TRY(ensure(c, c->bpart1, nb));
  }
  ST_TRY(ensure(c, c->alpha_part, (size_t)(Q / 16 + 64) * sizeof(double)));  // one per 16-pixel tile

  // PWLS runs on the device-resident loop only (P <= 48)
  const bool pwls = o->cost == CLSIMG_COST_PWLS;
  const bool device_loop = beam_fits(P) && outer_fits(P) && !c->old_beam && !c->host_loop && !c->trace;
  if (pwls && !device_loop) return CLSIMG_ENOTSUP;
  if (pwls && o->nsamples <= P + 1 && o->kappa_d != 0.0) return CLSIMG_EINVAL;
  if (pwls) {
    for (DevBuf* b : {&c->pw_h, &c->pw_rs, &c->pw_g, &c->pw_eps, &c->pw_dinv})
      ST_TRY(ensure(c, *b, (size_t)Q * sizeof(float)));
    ST_TRY(ensure(c, c->pw_Lw, (size_t)P * P * sizeof(float2)));
    ST_TRY(ensure(c, c->pw_B0w, (size_t)P * P * sizeof(float2)));
  }
  ST_TRY(ensure(c, c->eps, (size_t)Q * sizeof(float)));
  if (!mf_out) ST_TRY(ensure(c, c->mf, (size_t)Q * sizeof(float)));
  if (!gamma_out) ST_TRY(ensure(c, c->gamma, (size_t)Q * sizeof(float)));
  ST_TRY(ensure_tables(c, a, g, st));
  float* mf = mf_out ? mf_out : P_<float>(c->mf);
  float* gamma = gamma_out ? gamma_out : P_<float>(c->gamma);
  float* eps = P_<float>(c->eps);
  const float2* Rf = reinterpret_cast<const float2*>(R);
  float2* B0 = P_<float2>(c->B0);
  float2* Bb = P_<float2>(c->Bb);
  float2* u = P_<float2>(c->u);
  float2* E = P_<float2>(c->E);
  int* Flist = P_<int>(c->Flist);
  int* Ulist = P_<int>(c->Ulist);
  float* v = P_<float>(c->v);
  float* w = P_<float>(c->w);
  float* x = P_<float>(c->x);
  float* frag_r = P_<float>(c->frag_r);
  float* frag_u = P_<float>(c->frag_u);
  double* beta_part = P_<double>(c->beta_part);
  double* alpha_part = P_<double>(c->alpha_part);
  uint64_t* keys = P_<uint64_t>(c->keys);
  LsqrState* ls = P_<LsqrState>(c->lsqr);
  SolveDecision* dec = P_<SolveDecision>(c->dec);
  const int* lsqr_stop = &ls->done;
  const int* grad_stop = &dec->grad_done;
  const int nbeta = reduce_blocks(P);
  // fused two-kernel LSQR step for up to 12 row tiles (P <= 96)
  const int MT = pad_p(P) / 8;
  const bool fused = MT <= 12;
  const int nfw = lsqr_fwd_waves(P);
  LsqrState* S2 = P_<LsqrState>(c->lsqr2);
  LsqrState* Sfin = S2 + 2;
  int* done = P_<int>(c->done);
  float* x1 = P_<float>(c->x1);
  float* w1 = P_<float>(c->w1);
  float* vraw = P_<float>(c->vraw);
  double* bparts[2] = {P_<double>(c->bpart0), P_<double>(c->bpart1)};
  unsigned* bar = P_<unsigned>(c->bar);
  int* lerr = reinterpret_cast<int*>(bar + 1);
  float* xf = P_<float>(c->xf);

  double flops = beam_flops(P, Q) + (o->bound != CLSIMG_BOUND_NONE ? beam_flops(P, Q) : 0.0);
  // bounds and threshold (Sec. II-D, App. A)
  const float eps_scale = o->kappa_d != 0.0 ? (float)(o->kappa_d / sqrt((double)o->nsamples)) : 0.f;
  if (beam_any(P)) {
    ST_TRY(beam_full(c, g, P, Rf, BEAM_MF, mf, eps, eps_scale, 0, 0, 1.f, st));
  } else {
    HIP_TRY(launch_adjoint_mf(adj_params(c, g, P, nullptr, nullptr, Q, nullptr, Rf), mf, eps, eps_scale,
                              st));
  }
  ST_TRY(compute_bound(c, R, a, g, o, gamma, st));
  // data B0 = R - diag(noise), its norm, the starting image and sets
  HIP_TRY(launch_sub_diag(Rf, noise_diag, P, B0, st));
  ST_TRY(correlate(c, g, P, nullptr, nullptr, 0, 0, E, B0, 0.f, 1.f, nullptr, nullptr, beta_part,
                   nullptr, st));
  HIP_TRY(hipMemcpyAsync(c->h_norms, beta_part, nbeta * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(launch_init_state(sigma0, state0, sigma, state, Q, st));
  HIP_TRY(launch_compact(state, Q, Flist, Ulist, dec, st));
  ST_TRY(read_back(c, c->h_dec, dec, sizeof(SolveDecision), st));
  const double b0norm = sqrt(sum_host(c->h_norms, nbeta));
  int nF = c->h_dec->nF, nU = c->h_dec->nU;
  auto lsqr_adj = [&](const int* stop) {
    AdjParams a = adj_params(c, g, P, frag_u, Flist, nF, stop);
    a.xf = xf;
    return a;
  };
  // the LSQR adjoint of the split-K engine: for large arrays its rows are split
  // over workgroups, with the correlation's partial buffer (free by then) as
  // the workspace of the row groups' dots
  auto lsqr_adj_rows = [&](const int* stop) {
    AdjParams a = adj_params(c, g, P, frag_u, Flist, nF, stop);
    a.rows_part = P_<float>(c->part);
    a.rows_cap = c->part.bytes / sizeof(float);
    return a;
  };

  const int max_outer = o->max_outer < 0 ? 4 * Q : o->max_outer;
  int status = CLSIMG_OK;
  int outer = 0, adds = 0, drops = 0, lsqr_total = 0, itnlim_hits = 0, last_added = -1;
  bool need_solve = true;
  float lam_min = 0.f, eps_min = 0.f;
  int i_min = -1, st_min = 0;
  double margin_lambda = INFINITY, margin_z = INFINITY;
  int batch = 4;
  const int ntiles_Q = ntiles_adj(P, Q);
  const bool beam_full_grid = beam_fits(P) && !c->old_beam;
  // timing of the multiplier kernel (clsimg_kernel_timing): events bound to its launches
  const Stamps mult_stamps = c->time_mult ? Stamps{c->tm_ev[0], c->tm_ev[1]} : Stamps{};
  // reduced precision: the multipliers from one half-precision product, the
  // decision refined in FP32 over the candidates the rounding bound leaves
  const bool beam_half = c->prec != CLSIMG_FP32;
  const int cand_cap = std::max(64, std::min(Q / 8, kCandCap));
  const int cand_tile = adjoint_tile_width(MT);
  if (beam_half) {
    ST_TRY(ensure(c, c->frag_h, std::max(beam_h16_frag_bytes(P), beam_h1_frag_bytes(P))));
    ST_TRY(ensure(c, c->hscale, sizeof(float)));
    ST_TRY(ensure(c, c->mx_abs, kCandAbsParts * sizeof(double)));
    ST_TRY(ensure(c, c->mx_lam, (size_t)Q * sizeof(float)));
    ST_TRY(ensure(c, c->mx_cand, (size_t)cand_cap * sizeof(int)));
    ST_TRY(ensure(c, c->mx_count, sizeof(int)));
    const size_t nk = (size_t)std::max(beam_big_grid(P, Q, 2), (cand_cap + cand_tile - 1) / cand_tile) + 1;
    if (c->keys.bytes < nk * sizeof(uint64_t)) ST_TRY(ensure(c, c->keys, nk * sizeof(uint64_t)));
    keys = P_<uint64_t>(c->keys);
    const size_t rows = (size_t)((MT + 3) / 4) * 8 * cand_cap;  // row groups x K slices x list
    if (c->part.bytes < rows * sizeof(float)) ST_TRY(ensure(c, c->part, rows * sizeof(float)));
  }
  const bool beam_big_grid_ok = !beam_fits(P) && beam_big_fits(P) && !c->old_beam;
  bool host_loop = true;
  double dev_res2 = 0.0, dev_b0n2 = 0.0;  // residual of the device loop's last feasible step
  // PWLS inputs (eq. preWLS): Cholesky of R, h = a^H R^-1 a, D = h^2 / C, the
  // whitened data, bound D gamma and the MVDR-image threshold; the loop then
  // solves for D sigma
  const float* lam_scale = nullptr;
  const float* op_gamma = gamma;
  const float* op_eps = eps;
  const float2* op_B0 = B0;
  if (pwls) {
    if (o->bound != CLSIMG_BOUND_MVDR) {  // the MVDR bound has factorised R already
      HIP_TRY(launch_chol_inverse(Rf, P, P_<double2>(c->W), P_<double2>(c->Li), P_<float2>(c->Rinv),
                                  P_<int>(c->status), st));
      ST_TRY(read_back(c, c->h_status, c->status.ptr, sizeof(int), st));
      if (*c->h_status != 0) return CLSIMG_ENOTPD;
    }
    float* h = P_<float>(c->pw_h);
    ST_TRY(beam_full(c, g, P, P_<const float2>(c->Rinv), BEAM_STORE, h, nullptr, 0.f, 0, 0, 1.f, st));
    const double kd = o->kappa_d != 0.0 ? o->kappa_d / sqrt((double)(o->nsamples - P - 1)) : 0.0;
    HIP_TRY(launch_pwls_setup(h, gamma, o->C, kd, Q, P_<float>(c->pw_rs), P_<float>(c->pw_g),
                              P_<float>(c->pw_eps), P_<float>(c->pw_dinv), st));
    HIP_TRY(launch_pwls_whiten(P_<const double2>(c->Li), B0, P, P_<float2>(c->pw_Lw), P_<float2>(c->pw_B0w), st));
    if (sigma0) HIP_TRY(launch_pwls_scale(sigma, P_<const float>(c->pw_dinv), Q, true, st));  // D sigma0
    lam_scale = P_<const float>(c->pw_dinv);
    op_gamma = P_<const float>(c->pw_g);
    op_eps = P_<const float>(c->pw_eps);
    op_B0 = P_<const float2>(c->pw_B0w);
  }
  if (device_loop) {
    // Table I on the device: one workgroup per outer step, the full-grid
    // multiplier kernel between steps; the host only checks for the end
    OuterState* ost = P_<OuterState>(c->ostate);
    HIP_TRY(launch_outer_init(ost, dec, st));
    OuterParams op;
    op.st = ost;
    op.Flist = Flist;
    op.Ulist = Ulist;
    op.sigma = sigma;
    op.gamma = op_gamma;
    op.eps = op_eps;
    op.state = state;
    op.B0 = op_B0;
    op.Bb = Bb;
    op.E = E;
    op.keys = keys;
    op.nkeys = beam_grid(Q);
    op.tab = tables_of(c, g, P);
    op.P = P;
    op.Q = Q;
    op.atol = o->atol;
    op.btol = o->btol;
    op.conlim = o->conlim;
    op.itnlim = o->itnlim;
    op.max_outer = max_outer;
    op.max_f = c->outer_max_f;
    op.Lw = pwls ? P_<const float2>(c->pw_Lw) : nullptr;
    op.rowscale = pwls ? P_<const float>(c->pw_rs) : nullptr;
    int nb = 8;
    for (;;) {
      for (int b = 0; b < nb; ++b) {
        HIP_TRY(launch_outer_step(op, st));
        HIP_TRY(launch_beam_lambda(nullptr, E, P, op.tab, &ost->lam_skip, state, keys, lam_scale, st));
      }
      ST_TRY(read_back(c, c->h_outer, ost, sizeof(OuterState), st));
      if (c->h_outer->done) break;
      nb = std::min(2 * nb, 128);
    }
    const OuterState& S = *c->h_outer;
    status = S.status == kStatusMaxOuter ? CLSIMG_WMAXOUTER : (S.status == kStatusCycle ? CLSIMG_WCYCLE : CLSIMG_OK);
    outer = S.outer;
    adds = S.adds;
    drops = S.drops;
    lsqr_total = S.lsqr_total;
    itnlim_hits = S.itnlim_hits;
    last_added = S.last_added;
    margin_lambda = S.margin_lambda;
    margin_z = S.margin_z;
    nF = S.nF;
    nU = S.nU;
    flops += S.psi_flops;
    // a free set too large for one workgroup: continue on the host from here
    host_loop = S.fallback != 0;
    dev_res2 = S.res2;
    dev_b0n2 = S.b0n2;
    if (pwls) {
      if (host_loop) return CLSIMG_ENOTSUP;  // the host loop has no PWLS path
      HIP_TRY(launch_pwls_scale(sigma, P_<const float>(c->pw_dinv), Q, false, st));  // sigma = D^-1 (D sigma)
    }
  }
  for (; host_loop;) {
    if (need_solve) {
      if (outer >= max_outer) {
        status = CLSIMG_WMAXOUTER;
        break;
      }
      HIP_TRY(launch_compact(state, Q, Flist, Ulist, dec, st));
      // b = B0 - Psi_U gamma_U  (eq. bsubproblemLS); b = B0 while U is empty
      const float2* bsub = B0;
      if (nU > 0) {
        ST_TRY(correlate(c, g, P, Ulist, gamma, 1, nU, Bb, B0, -1.f, 1.f, nullptr, nullptr, nullptr,
                         nullptr, st));
        bsub = Bb;
      }
      flops += corr_flops(P, nU);
      if (fused) {
        // the cache grows geometrically with |F| (a reallocation synchronises the device)
        size_t cap = 256;
        while (cap < (size_t)nF) cap *= 2;
        ST_TRY(ensure(c, c->xf, cap * 2 * pad_p(P) * sizeof(float)));
        xf = P_<float>(c->xf);
        HIP_TRY(launch_xf(tables_of(c, g, P), Flist, nF, xf, st));
      }
      const int nalpha = ntiles_adj(P, nF);
      const int nalpha2 = (nF + adjoint_lsqr2_tile_width(MT, nF) - 1) / adjoint_lsqr2_tile_width(MT, nF);
      int it = 1;
      auto fwd_params = [&](int iter) {
        LsqrFwdParams f;
        f.tab = tables_of(c, g, P);
        f.MT = MT;
        f.P = P;
        f.Flist = Flist;
        f.n = nF;
        f.S = S2;
        f.Sfinal = Sfin;
        f.done = done;
        f.it = iter;
        f.vraw = vraw;
        f.vnorm = v;
        f.alpha_part = alpha_part;
        f.nalpha = nalpha2;
        f.beta_in = bparts[iter & 1];
        f.nbeta_in = iter == 1 ? nbeta : nfw;
        f.beta_out = bparts[(iter + 1) & 1];
        f.x0 = x;
        f.x1 = x1;
        f.w0 = w;
        f.w1 = w1;
        f.xf = xf;
        f.u = u;
        f.frag = frag_u;
        f.ntp = MT * (MT + 1) / 2;
        return f;
      };
      // LSQR engine: one workgroup when the subproblem fits in its LDS (no grid
      // barriers at all), else one cooperative kernel, else two kernels per
      // step (P <= 96), else the split-K correlation with separate reductions
      const int want = c->lsqr_path;
      const bool one_cu = fused && (want == 0 || want == 1) && lsqr_cu_fits(P, nF);
      const bool persist = !one_cu && fused && c->coop && (want == 0 || want == 2) && persist_fits(P, nF);
      if (nF > 0) {
        const int itnlim = o->itnlim < 0 ? 4 * nF + 100 : o->itnlim;
        if (one_cu) {
          HIP_TRY(launch_lsqr_setup2(S2, done, bar, lerr, o->atol, o->btol, o->conlim, itnlim, st));
          LsqrCuParams lc;
          lc.P = P;
          lc.n = nF;
          lc.xf = xf;
          lc.B = bsub;
          lc.x_out = x;
          lc.Sfinal = Sfin;
          lc.done = done;
          lc.atol = o->atol;
          lc.btol = o->btol;
          lc.conlim = o->conlim;
          lc.itnlim = itnlim;
          HIP_TRY(launch_lsqr_cu(lc, st));
        } else if (persist) {
          // the whole LSQR solve in one cooperative kernel
          HIP_TRY(launch_lsqr_setup2(S2, done, bar, lerr, o->atol, o->btol, o->conlim, itnlim, st));
          LsqrPersistParams lp;
          lp.MT = MT;
          lp.P = P;
          lp.n = nF;
          lp.ntp = MT * (MT + 1) / 2;
          lp.xf = xf;
          lp.B = bsub;
          lp.frag = frag_u;
          lp.pbeta = bparts[0];
          lp.palpha = alpha_part;
          lp.vraw = vraw;
          lp.x_out = x;
          lp.Sfinal = Sfin;
          lp.done = done;
          lp.bar = bar;
          lp.err = lerr;
          lp.atol = o->atol;
          lp.btol = o->btol;
          lp.conlim = o->conlim;
          lp.itnlim = itnlim;
          HIP_TRY(launch_lsqr_persist(lp, st));
        } else if (fused) {
          // beta_1 u_1 = b ; alpha_1 v_1 = Psi_F^H u_1  (eqs. initbeta, initu); then step 1
          HIP_TRY(launch_lsqr_setup(S2, done, o->atol, o->btol, o->conlim, itnlim, st));
          ST_TRY(correlate(c, g, P, nullptr, nullptr, 0, 0, u, bsub, 0.f, 1.f, nullptr, frag_u,
                           bparts[1], nullptr, st));
          HIP_TRY(launch_adjoint_lsqr2(lsqr_adj(done), EpiLsqrV2{vraw, v, bparts[1], nbeta, alpha_part, 1},
                                       st));
          HIP_TRY(launch_lsqr_fwd(fwd_params(1), st));
        } else {
          ST_TRY(correlate(c, g, P, nullptr, nullptr, 0, 0, u, bsub, 0.f, 1.f, nullptr, frag_u, beta_part,
                           nullptr, st));
          HIP_TRY(launch_adjoint_lsqr(lsqr_adj_rows(nullptr), v, beta_part, nbeta, alpha_part, 1, st));
          HIP_TRY(launch_lsqr_init_scalars(ls, beta_part, nbeta, alpha_part, nalpha, v, w, x, nF,
                                           o->atol, o->btol, o->conlim, itnlim, st));
        }
      }
      for (;;) {
        if (nF > 0 && !persist && !one_cu) {
          for (int b = 0; b < batch; ++b) {
            // beta u <- Psi_F v - alpha u ; alpha v <- Psi_F^H u - beta v  (eq. lanczos)
            if (fused) {
              HIP_TRY(launch_adjoint_lsqr2(lsqr_adj(done),
                                           EpiLsqrV2{vraw, v, bparts[(it + 1) & 1], nfw, alpha_part, 0},
                                           st));
              ++it;
              HIP_TRY(launch_lsqr_fwd(fwd_params(it), st));
            } else {
              ST_TRY(correlate(c, g, P, Flist, v, 0, nF, u, u, 1.f, 0.f, ls, frag_u, beta_part,
                               lsqr_stop, st));
              HIP_TRY(launch_adjoint_lsqr(lsqr_adj_rows(lsqr_stop), v, beta_part, nbeta, alpha_part, 0, st));
              HIP_TRY(launch_lsqr_update(ls, beta_part, nbeta, alpha_part, nalpha, v, w, x, nF, st));
            }
          }
        }
        if (persist || one_cu)
          HIP_TRY(launch_step(done, lerr, Sfin, x, x, Flist, nF, sigma, gamma, state, dec, st));
        else if (fused)
          HIP_TRY(launch_step(done, nullptr, Sfin, x, x1, Flist, nF, sigma, gamma, state, dec, st));
        else
          HIP_TRY(launch_step(lsqr_stop, nullptr, ls, x, x, Flist, nF, sigma, gamma, state, dec, st));
        // gradient on the active pixels, only after a feasible subproblem (eq. gls):
        // E = Psi_F sigma_F - b, then g = Psi^H E on every pixel
        if (fused) {
          CorrOsParams cp;
          cp.MT = MT;
          cp.P = P;
          cp.xf = xf;
          cp.n = nF;
          cp.vals = sigma;
          cp.gidx = Flist;
          cp.out = E;
          cp.B = bsub;
          cp.cK = 1.f;
          cp.cB = -1.f;
          cp.frag = frag_r;
          cp.stop_flag = grad_stop;
          HIP_TRY(launch_corr_os(cp, st));
        } else {
          ST_TRY(correlate(c, g, P, Flist, sigma, 1, nF, E, bsub, 1.f, -1.f, nullptr, frag_r, nullptr,
                           grad_stop, st));
        }
        if (beam_half) {
          const bool bf = c->prec == CLSIMG_BF16;
          int* count = P_<int>(c->mx_count);
          HIP_TRY(launch_beam_lambda_refined(E, P, bf, tables_of(c, g, P), grad_stop, state, c->frag_h.ptr,
                                             P_<float>(c->hscale), P_<double>(c->mx_abs), kCandAbsParts, keys,
                                             P_<float>(c->mx_lam), P_<int>(c->mx_cand), cand_cap, count, st,
                                             big_tiles(c, P), mult_stamps));
          // the candidates in FP32: Ut fragments of E from the correlation
          AdjParams ap = adj_params(c, g, P, frag_r, P_<const int>(c->mx_cand), cand_cap, grad_stop);
          ap.rows_part = P_<float>(c->part);
          ap.rows_cap = c->part.bytes / sizeof(float);
          ap.n_dev = count;
          HIP_TRY(launch_adjoint_lambda(ap, state, keys, st));
          HIP_TRY(launch_argmin_final(keys, (cand_cap + cand_tile - 1) / cand_tile, eps, state, dec, st, count,
                                      cand_cap));
        } else if (!beam_full_grid && beam_big_grid_ok) {
          HIP_TRY(launch_beam_prep_full(E, P, P_<float>(c->frag_b), st));
          HIP_TRY(launch_beam_big(3, P_<const float>(c->frag_b), tables_of(c, g, P), grad_stop, nullptr, nullptr, 0.f,
                                  0, 0, 1.f, state, keys, st, mult_stamps, big_tiles(c, P)));
          HIP_TRY(launch_argmin_final(keys, beam_big_grid(P, Q, big_tiles(c, P)), eps, state, dec, st));
        } else if (beam_full_grid) {
          if (c->beam_prep) HIP_TRY(launch_beam_prep(E, P, P_<float>(c->frag_b), st));
          HIP_TRY(launch_beam_lambda(c->beam_prep ? P_<const float>(c->frag_b) : nullptr,
                                     c->beam_prep ? nullptr : E, P, tables_of(c, g, P), grad_stop, state,
                                     keys, nullptr, st));
          HIP_TRY(launch_argmin_final(keys, beam_grid(Q), eps, state, dec, st));
        } else {
          HIP_TRY(launch_adjoint_lambda(adj_params(c, g, P, frag_r, nullptr, Q, grad_stop), state, keys,
                                        st));
          HIP_TRY(launch_argmin_final(keys, ntiles_Q, eps, state, dec, st));
        }
        ST_TRY(read_back(c, c->h_dec, dec, sizeof(SolveDecision), st));
        if (mult_stamps.start && c->h_dec->lsqr_done && c->h_dec->feasible && (beam_half || !beam_full_grid)) {
          float ms = 0.f;
          HIP_TRY(hipEventElapsedTime(&ms, c->tm_ev[0], c->tm_ev[1]));
          c->tm_ms += ms;
          ++c->tm_n;
        }
        if (beam_half && c->h_dec->lsqr_done && c->h_dec->feasible && c->h_dec->cand_overflow) {
          // more candidates than the list holds: this step's multipliers in FP32
          if (beam_full_grid) {
            HIP_TRY(launch_beam_lambda(nullptr, E, P, tables_of(c, g, P), grad_stop, state, keys, nullptr, st));
            HIP_TRY(launch_argmin_final(keys, beam_grid(Q), eps, state, dec, st));
          } else if (beam_big_grid_ok) {
            HIP_TRY(launch_beam_prep_full(E, P, P_<float>(c->frag_b), st));
            HIP_TRY(launch_beam_big(3, P_<const float>(c->frag_b), tables_of(c, g, P), grad_stop, nullptr, nullptr,
                                    0.f, 0, 0, 1.f, state, keys, st, {}, big_tiles(c, P)));
            HIP_TRY(launch_argmin_final(keys, beam_big_grid(P, Q, big_tiles(c, P)), eps, state, dec, st));
          } else {
            HIP_TRY(launch_adjoint_lambda(adj_params(c, g, P, frag_r, nullptr, Q, grad_stop), state, keys, st));
            HIP_TRY(launch_argmin_final(keys, ntiles_Q, eps, state, dec, st));
          }
          ST_TRY(read_back(c, c->h_dec, dec, sizeof(SolveDecision), st));
          if (c->trace) fprintf(stderr, "clsimg: outer %d: candidate list full, multipliers in FP32\n", outer);
        }
        if (c->h_dec->lsqr_done) break;
        if (persist || one_cu || c->h_dec->lsqr_err) return CLSIMG_EHIP;  // LSQR kernel did not finish
        batch = std::min(batch * 2, 64);
      }
      const SolveDecision d = *c->h_dec;
      if (c->trace) {
        ST_TRY(read_back(c, c->h_lsqr, fused ? Sfin : ls, sizeof(LsqrState), st));
        const LsqrState& L = *c->h_lsqr;
        fprintf(stderr,
                "clsimg: outer %d nF %d nU %d itn %d istop %d alpha %.3e beta %.3e rnorm %.3e "
                "arnorm %.3e anorm %.3e acond %.3e xnorm %.3e bnorm %.3e feasible %d ib %d mu %.3e "
                "i_min %d lam %.4e eps %.4e\n",
                outer, nF, nU, L.itn, L.istop, L.alpha, L.beta, L.rnorm, L.arnorm, L.anorm, L.acond,
                L.xnorm, L.bnorm, d.feasible, d.ib, (double)d.mu_max, d.i_min, (double)d.lam_min,
                (double)d.eps_min);
      }
      batch = std::max(2, std::min(64, d.lsqr_itn + 1));
      ++outer;
      lsqr_total += d.lsqr_itn;
      if (nF > 0) flops += beam_flops(P, nF) + d.lsqr_itn * (corr_flops(P, nF) + beam_flops(P, nF));
      if (d.feasible) flops += corr_flops(P, nF) + beam_flops(P, Q);
      if (nF > 0 && d.lsqr_istop == 7) ++itnlim_hits;
      if (d.feasible) {
        need_solve = false;
        if (nF > 0) margin_z = std::min(margin_z, (double)d.margin_z);
        if (d.i_min < 0) break;  // no active pixel left
        lam_min = d.lam_min;
        eps_min = d.eps_min;
        i_min = d.i_min;
        st_min = d.st_min;
      } else {
        ++drops;
        --nF;
        if (d.ib_to == CLSIMG_STATE_U) ++nU;
        need_solve = true;
        if (d.ib == last_added && d.mu_max == 0.0f) {
          status = CLSIMG_WCYCLE;
          break;
        }
      }
      last_added = -1;
    } else {
      if (eps_min > 0.f)
        margin_lambda = std::min(margin_lambda, fabs((double)lam_min + eps_min) / eps_min);
      if (lam_min < -eps_min) {
        HIP_TRY(launch_set_state(state, i_min, (uint8_t)CLSIMG_STATE_F, st));
        ++adds;
        ++nF;
        if (st_min == CLSIMG_STATE_U) --nU;
        last_added = i_min;
        need_solve = true;
      } else {
        break;
      }
    }
  }
  if (status == CLSIMG_OK && itnlim_hits) status = CLSIMG_WITNLIM;
  if (!host_loop) {
    // finished on the device: the residual of the last feasible step (the
    // final image), as the batched and served solves report it
    stats->status = status;
    stats->outer_iters = outer;
    stats->adds = adds;
    stats->drops = drops;
    stats->lsqr_iters_total = lsqr_total;
    stats->lsqr_itnlim_hits = itnlim_hits;
    stats->nF = nF;
    stats->nU = nU;
    stats->rel_residual = dev_b0n2 > 0.0 ? sqrt(dev_res2 / dev_b0n2) : 0.0;
    stats->objective = 0.5 * dev_res2;
    stats->min_margin_lambda = margin_lambda;
    stats->min_margin_z = margin_z;
    stats->psi_flops = flops;
    return status;
  }
  // final residual ||B0 - Psi sigma||_F
  HIP_TRY(launch_compact(state, Q, Flist, Ulist, dec, st));
  ST_TRY(read_back(c, c->h_dec, dec, sizeof(SolveDecision), st));
  nF = c->h_dec->nF;
  nU = c->h_dec->nU;
  ST_TRY(correlate(c, g, P, Ulist, gamma, 1, nU, Bb, B0, -1.f, 1.f, nullptr, nullptr, nullptr, nullptr,
                   st));
  ST_TRY(correlate(c, g, P, Flist, sigma, 1, nF, E, Bb, 1.f, -1.f, nullptr, nullptr, beta_part,
                   nullptr, st));
  ST_TRY(read_back(c, c->h_norms, beta_part, nbeta * sizeof(double), st));
  const double rn = sqrt(sum_host(c->h_norms, nbeta));
  stats->status = status;
  stats->outer_iters = outer;
  stats->adds = adds;
  stats->drops = drops;
  stats->lsqr_iters_total = lsqr_total;
  stats->lsqr_itnlim_hits = itnlim_hits;
  stats->nF = nF;
  stats->nU = nU;
  stats->rel_residual = b0norm > 0 ? rn / b0norm : 0.0;
  stats->objective = 0.5 * rn * rn;
  stats->min_margin_lambda = margin_lambda;
  stats->min_margin_z = margin_z;
  stats->psi_flops = flops + corr_flops(P, nU) + corr_flops(P, nF);
  return status;
}

// K covariance blocks over one grid (eq. vectRtotal): the host-driven
// active-set loop of clsimg_solve with every operator applied per block --
// the correlations give one matrix per block, the beamformer outputs are
// summed over the blocks (stacked Khatri-Rao operator), and the images, the
// bound and the multipliers come from the block sums (eqs. mfdimg, wmvdr,
// App. A; gradient (1/K) sum_k, eq. UCLS).  LSQR runs on the stacked blocks
// with the split-K correlation and the LDS-staged adjoint, each launched
// once for all blocks.
namespace {
struct TableOverride {
  clsimg_ctx* c;
  ~TableOverride() {
    c->tab_El = nullptr;
    c->tab_Em = nullptr;
  }
};
}  // namespace

int clsimg_solve_multi(clsimg_ctx* c, int32_t K, const clsimg_block* blocks, const clsimg_grid* g,
                       const clsimg_opts* o, float* sigma, uint8_t* state, float* mf_out, float* gamma_out,
                       clsimg_stats* stats, void* stream) {
  if (stats) memset(stats, 0, sizeof(*stats));
  if (!c || !blocks || K < 1 || K > CLSIMG_MAX_BLOCKS || !g || !sigma || !state || !stats) return CLSIMG_EINVAL;
  const int P = blocks[0].array.P;
  for (int k = 0; k < K; ++k) {
    if (!blocks[k].R || blocks[k].array.P != P) return CLSIMG_EINVAL;
    ST_TRY(check_geometry(&blocks[k].array, g));
  }
  ST_TRY(check_opts(o, P));
  if (o->nsamples <= 0 && o->kappa_d != 0.0) return CLSIMG_EINVAL;
  if (o->cost != CLSIMG_COST_LS) return CLSIMG_ENOTSUP;
  c->prec = o->precision;
  DeviceGuard guard(c->device);
  hipStream_t st = (hipStream_t)stream;
  TableOverride restore{c};
  const int Q = g->nl * g->nm, Pp = pad_p(P), MT = Pp / 8;
  const int nl = g->nl, nm = g->nm;
  ST_TRY(ensure_workspace(c, P, Q));
  const int nbeta = reduce_blocks(P);
  const size_t cx = (size_t)P * P * sizeof(float2);
  const size_t tab_b = (size_t)Pp * (nl + nm) * sizeof(float2);
  const size_t fru = (size_t)4 * Pp * Pp;  // fragment floats of one block's u
  ST_TRY(ensure(c, c->mb_tab, K * tab_b));
  ST_TRY(ensure(c, c->mb_B0, K * cx));
  ST_TRY(ensure(c, c->mb_Bb, K * cx));
  ST_TRY(ensure(c, c->mb_u, K * cx));
  ST_TRY(ensure(c, c->mb_E, K * cx));
  ST_TRY(ensure(c, c->mb_frag, K * fru * sizeof(float)));
  ST_TRY(ensure(c, c->mb_acc, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->mb_acc2, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->part, (size_t)K * part_floats_max(P) * sizeof(float)));
  // the lists and LSQR vectors of the host-driven loop (not part of the common workspace)
  ST_TRY(ensure(c, c->Flist, (size_t)Q * sizeof(int)));
  ST_TRY(ensure(c, c->Ulist, (size_t)Q * sizeof(int)));
  ST_TRY(ensure(c, c->v, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->w, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->x, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->beta_part, (size_t)K * nbeta * sizeof(double)));
  ST_TRY(ensure(c, c->eps, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->alpha_part, (size_t)(Q / 16 + 64) * sizeof(double)));
  if (!mf_out) ST_TRY(ensure(c, c->mf, (size_t)Q * sizeof(float)));
  if (!gamma_out) ST_TRY(ensure(c, c->gamma, (size_t)Q * sizeof(float)));
  if (c->prec != CLSIMG_FP32) {
    ST_TRY(ensure(c, c->frag_h, beam_h16_frag_bytes(P)));
    ST_TRY(ensure(c, c->hscale, sizeof(float)));
  }
  if ((size_t)K * nbeta > c->h_mnorm_n) {
    HIP_TRY(hipStreamSynchronize(st));
    if (c->h_mnorm) (void)hipHostFree(c->h_mnorm);
    c->h_mnorm = nullptr;
    c->h_mnorm_n = 0;
    HIP_TRY(hipHostMalloc((void**)&c->h_mnorm, (size_t)K * nbeta * sizeof(double), hipHostMallocDefault));
    c->h_mnorm_n = (size_t)K * nbeta;
  }
  float* mf = mf_out ? mf_out : P_<float>(c->mf);
  float* gamma = gamma_out ? gamma_out : P_<float>(c->gamma);
  float* eps = P_<float>(c->eps);
  float* acc = P_<float>(c->mb_acc);
  float* acc2 = P_<float>(c->mb_acc2);
  double* beta_part = P_<double>(c->beta_part);
  double* alpha_part = P_<double>(c->alpha_part);
  uint64_t* keys = P_<uint64_t>(c->keys);
  LsqrState* ls = P_<LsqrState>(c->lsqr);
  SolveDecision* dec = P_<SolveDecision>(c->dec);
  const int* lsqr_stop = &ls->done;
  const int* grad_stop = &dec->grad_done;
  int* Flist = P_<int>(c->Flist);
  int* Ulist = P_<int>(c->Ulist);
  float* v = P_<float>(c->v);
  float* w = P_<float>(c->w);
  float* x = P_<float>(c->x);
  auto B0k = [&](int k) { return P_<float2>(c->mb_B0) + (size_t)k * P * P; };
  auto Bbk = [&](int k) { return P_<float2>(c->mb_Bb) + (size_t)k * P * P; };
  auto uk = [&](int k) { return P_<float2>(c->mb_u) + (size_t)k * P * P; };
  auto Ek = [&](int k) { return P_<float2>(c->mb_E) + (size_t)k * P * P; };
  auto fragk = [&](int k) { return P_<float>(c->mb_frag) + (size_t)k * fru; };
  // steering tables of every block, kept side by side
  for (int k = 0; k < K; ++k) {
    c->tab_El = nullptr;
    c->tab_Em = nullptr;
    ST_TRY(ensure_tables(c, &blocks[k].array, g, st));
    char* tb = P_<char>(c->mb_tab) + (size_t)k * tab_b;
    HIP_TRY(hipMemcpyAsync(tb, c->El.ptr, (size_t)Pp * nl * sizeof(float2), hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(tb + (size_t)Pp * nl * sizeof(float2), c->Em.ptr, (size_t)Pp * nm * sizeof(float2),
                           hipMemcpyDeviceToDevice, st));
  }
  auto use = [&](int k) {
    const float2* tb = reinterpret_cast<const float2*>(P_<char>(c->mb_tab) + (size_t)k * tab_b);
    c->tab_El = tb;
    c->tab_Em = tb + (size_t)Pp * nl;
  };
  const size_t tstride = tab_b / sizeof(float2), pp2 = (size_t)P * P;
  // one correlation launch pair for all blocks: block k at k * stride
  auto corr = [&](const int* idx, const float* vals, int gather, int n, float2* out, const float2* B, float cK,
                  float cB, const LsqrState* lsq, float* frag, double* norms, const int* stop) {
    use(0);
    return correlate_blocks(c, g, P, K, tstride, idx, vals, gather, n, out, pp2, B, pp2, cK, cB, lsq, frag,
                            frag ? fru : 0, norms, norms ? (size_t)nbeta : 0, stop, st);
  };
  auto beam_acc = [&](int k, const float2* U, const int* skip, float* sum, float* sumsq, float scale) {
    use(k);
    return launch_beam_accumulate(U, P, tables_of(c, g, P), skip, sum, sumsq, scale, k == 0, c->prec,
                                  P_<float>(c->frag_b), c->frag_h.ptr, P_<float>(c->hscale), st, big_tiles(c, P));
  };
  const double Kd = K;
  double flops = 0.0;
  // MF image and threshold (eq. mfdimg, App. A)
  for (int k = 0; k < K; ++k)
    HIP_TRY(beam_acc(k, reinterpret_cast<const float2*>(blocks[k].R), nullptr, mf, acc2, (float)(1.0 / Kd)));
  flops += K * beam_flops(P, Q);
  const double sqn = o->nsamples > 0 ? sqrt((double)o->nsamples) : 1.0;
  HIP_TRY(launch_multi_mf(acc2, Q, (float)(o->kappa_d / (Kd * sqn)), eps, st));
  // bound (eq. wmvdr with the sqrt(K) normalisation, Sec. II-D, App. A)
  if (o->bound == CLSIMG_BOUND_NONE) {
    HIP_TRY(launch_fill(gamma, std::numeric_limits<float>::infinity(), Q, st));
  } else if (o->bound == CLSIMG_BOUND_MF) {
    HIP_TRY(launch_multi_bound(1, mf, acc2, Q, 0.0, Kd, o->kappa_b / (Kd * sqn), gamma, st));
  } else {
    for (int k = 0; k < K; ++k) {
      HIP_TRY(launch_chol_inverse(reinterpret_cast<const float2*>(blocks[k].R), P, P_<double2>(c->W),
                                  P_<double2>(c->Li), P_<float2>(c->Rinv), P_<int>(c->status), st));
      ST_TRY(read_back(c, c->h_status, c->status.ptr, sizeof(int), st));
      if (*c->h_status != 0) return CLSIMG_ENOTPD;
      HIP_TRY(beam_acc(k, P_<const float2>(c->Rinv), nullptr, acc, acc2, 1.f));
    }
    flops += K * beam_flops(P, Q);
    const double kb = o->kappa_b != 0.0 ? o->kappa_b / sqrt((double)(o->nsamples - P - 1)) : 0.0;
    HIP_TRY(launch_multi_bound(0, acc, acc2, Q, o->C, Kd, kb, gamma, st));
  }
  // data B0_k = R_k - diag(noise_k) and ||B0||
  for (int k = 0; k < K; ++k)
    HIP_TRY(launch_sub_diag(reinterpret_cast<const float2*>(blocks[k].R), blocks[k].noise_diag, P, B0k(k), st));
  ST_TRY(corr(nullptr, nullptr, 0, 0, Ek(0), B0k(0), 0.f, 1.f, nullptr, nullptr, beta_part, nullptr));
  ST_TRY(read_back(c, c->h_mnorm, beta_part, (size_t)K * nbeta * sizeof(double), st));
  const double b0norm = sqrt(sum_host(c->h_mnorm, K * nbeta));
  HIP_TRY(launch_init_state(nullptr, nullptr, sigma, state, Q, st));
  HIP_TRY(launch_compact(state, Q, Flist, Ulist, dec, st));
  ST_TRY(read_back(c, c->h_dec, dec, sizeof(SolveDecision), st));
  int nF = c->h_dec->nF, nU = c->h_dec->nU;

  const int max_outer = o->max_outer < 0 ? 4 * Q : o->max_outer;
  const int nkeys = lambda_vec_blocks(Q);
  int status = CLSIMG_OK;
  int outer = 0, adds = 0, drops = 0, lsqr_total = 0, itnlim_hits = 0, last_added = -1;
  bool need_solve = true;
  float lam_min = 0.f, eps_min = 0.f;
  int i_min = -1, st_min = 0;
  double margin_lambda = INFINITY, margin_z = INFINITY;
  int batch = 2;
  for (;;) {
    if (need_solve) {
      if (outer >= max_outer) {
        status = CLSIMG_WMAXOUTER;
        break;
      }
      HIP_TRY(launch_compact(state, Q, Flist, Ulist, dec, st));
      // b_k = B0_k - Psi_{U,k} gamma_U  (eq. bsubproblemLS per block)
      ST_TRY(corr(Ulist, gamma, 1, nU, Bbk(0), B0k(0), -1.f, 1.f, nullptr, nullptr, nullptr, nullptr));
      flops += K * corr_flops(P, nU);
      const int nalpha = (nF + 63) / 64;  // the 64-column tiles of launch_lsqr_v_blocks
      const int itnlim = o->itnlim < 0 ? 4 * nF + 100 : o->itnlim;
      // Psi_F^H u over the blocks: one launch whose workgroup rows are the
      // blocks (column dots kept apart), then the LSQR v update adds them in
      // block order
      if (nF > 0) ST_TRY(ensure(c, c->mb_gpart, (size_t)K * nF * sizeof(float)));
      auto adjoint_all = [&](int init, const int* stop) -> int {
        use(0);
        AdjParams ap = adj_params(c, g, P, fragk(0), Flist, nF, stop);
        ap.nblk = K;
        ap.frag_stride = fru;
        ap.tab_stride = tstride;
        HIP_TRY(launch_adjoint_store_blocks(ap, P_<float>(c->mb_gpart), (size_t)nF, st));
        HIP_TRY(launch_lsqr_v_blocks(P_<const float>(c->mb_gpart), K, (size_t)nF, nF, v, beta_part, K * nbeta,
                                     alpha_part, init, stop, st));
        return CLSIMG_OK;
      };
      if (nF > 0) {
        // beta_1 u_1 = b ; alpha_1 v_1 = Psi_F^H u_1  (eqs. initbeta, initu)
        ST_TRY(corr(nullptr, nullptr, 0, 0, uk(0), Bbk(0), 0.f, 1.f, nullptr, fragk(0), beta_part, nullptr));
        ST_TRY(adjoint_all(1, nullptr));
        HIP_TRY(launch_lsqr_init_scalars(ls, beta_part, K * nbeta, alpha_part, nalpha, v, w, x, nF, o->atol,
                                         o->btol, o->conlim, itnlim, st));
      }
      for (;;) {
        if (nF > 0) {
          for (int b = 0; b < batch; ++b) {
            // beta u <- Psi_F v - alpha u ; alpha v <- Psi_F^H u - beta v  (eq. lanczos), all blocks
            ST_TRY(corr(Flist, v, 0, nF, uk(0), uk(0), 1.f, 0.f, ls, fragk(0), beta_part, lsqr_stop));
            ST_TRY(adjoint_all(0, lsqr_stop));
            HIP_TRY(launch_lsqr_update(ls, beta_part, K * nbeta, alpha_part, nalpha, v, w, x, nF, st));
          }
        }
        HIP_TRY(launch_step(lsqr_stop, nullptr, ls, x, x, Flist, nF, sigma, gamma, state, dec, st));
        // gradient after a feasible subproblem (eq. gls, cost of eq. UCLS):
        // E_k = Psi_{F,k} sigma_F - b_k, g = (1/K) sum_k vectdiag(A_k^H E_k A_k)
        ST_TRY(corr(Flist, sigma, 1, nF, Ek(0), Bbk(0), 1.f, -1.f, nullptr, nullptr, nullptr, grad_stop));
        for (int k = 0; k < K; ++k) HIP_TRY(beam_acc(k, Ek(k), grad_stop, acc2, nullptr, (float)(1.0 / Kd)));
        HIP_TRY(launch_lambda_vec(acc2, state, Q, grad_stop, keys, st));
        HIP_TRY(launch_argmin_final(keys, nkeys, eps, state, dec, st));
        ST_TRY(read_back(c, c->h_dec, dec, sizeof(SolveDecision), st));
        if (c->h_dec->lsqr_done) break;
        batch = std::min(batch * 2, 64);
      }
      const SolveDecision d = *c->h_dec;
      batch = std::max(2, std::min(64, d.lsqr_itn + 1));
      ++outer;
      lsqr_total += d.lsqr_itn;
      if (nF > 0) flops += K * (beam_flops(P, nF) + d.lsqr_itn * (corr_flops(P, nF) + beam_flops(P, nF)));
      if (d.feasible) flops += K * (corr_flops(P, nF) + beam_flops(P, Q));
      if (nF > 0 && d.lsqr_istop == 7) ++itnlim_hits;
      if (d.feasible) {
        need_solve = false;
        if (nF > 0) margin_z = std::min(margin_z, (double)d.margin_z);
        if (d.i_min < 0) break;  // no active pixel left
        lam_min = d.lam_min;
        eps_min = d.eps_min;
        i_min = d.i_min;
        st_min = d.st_min;
      } else {
        ++drops;
        --nF;
        if (d.ib_to == CLSIMG_STATE_U) ++nU;
        need_solve = true;
        if (d.ib == last_added && d.mu_max == 0.0f) {
          status = CLSIMG_WCYCLE;
          break;
        }
      }
      last_added = -1;
    } else {
      if (eps_min > 0.f) margin_lambda = std::min(margin_lambda, fabs((double)lam_min + eps_min) / eps_min);
      if (lam_min < -eps_min) {
        HIP_TRY(launch_set_state(state, i_min, (uint8_t)CLSIMG_STATE_F, st));
        ++adds;
        ++nF;
        if (st_min == CLSIMG_STATE_U) --nU;
        last_added = i_min;
        need_solve = true;
      } else {
        break;
      }
    }
  }
  if (status == CLSIMG_OK && itnlim_hits) status = CLSIMG_WITNLIM;
  // final residual sum_k ||B0_k - Psi_k sigma||^2
  HIP_TRY(launch_compact(state, Q, Flist, Ulist, dec, st));
  ST_TRY(read_back(c, c->h_dec, dec, sizeof(SolveDecision), st));
  nF = c->h_dec->nF;
  nU = c->h_dec->nU;
  ST_TRY(corr(Ulist, gamma, 1, nU, Bbk(0), B0k(0), -1.f, 1.f, nullptr, nullptr, nullptr, nullptr));
  ST_TRY(corr(Flist, sigma, 1, nF, Ek(0), Bbk(0), 1.f, -1.f, nullptr, nullptr, beta_part, nullptr));
  ST_TRY(read_back(c, c->h_mnorm, beta_part, (size_t)K * nbeta * sizeof(double), st));
  const double rn = sqrt(sum_host(c->h_mnorm, K * nbeta));
  stats->status = status;
  stats->outer_iters = outer;
  stats->adds = adds;
  stats->drops = drops;
  stats->lsqr_iters_total = lsqr_total;
  stats->lsqr_itnlim_hits = itnlim_hits;
  stats->nF = nF;
  stats->nU = nU;
  stats->rel_residual = b0norm > 0 ? rn / b0norm : 0.0;
  stats->objective = 0.5 * rn * rn / Kd;
  stats->min_margin_lambda = margin_lambda;
  stats->min_margin_z = margin_z;
  stats->psi_flops = flops + K * (corr_flops(P, nU) + corr_flops(P, nF));
  (void)MT;
  return status;
}

// Strong off-grid sources (Sec. III-E, eq. doals): the host-driven active-set
// loop with the subproblem replaced by rounds of (LSQR on the free pixels at
// their shifted directions, one Gauss-Newton step per free pixel's offset),
// then a final LSQR; the free pixels' bounds are taken at their shifted
// directions; the upper set keeps on-grid steering and bounds; release tests
// and the gradient on the active pixels stay on the grid.  P <= 48 and free
// sets within the one-workgroup LSQR.
int clsimg_solve_offgrid(clsimg_ctx* c, const clsimg_c32* R, const clsimg_array* a, const clsimg_grid* g,
                         const float* noise_diag, const clsimg_opts* o, int32_t rounds, float* sigma,
                         uint8_t* state, float* offsets, float* mf_out, float* gamma_out, clsimg_stats* stats,
                         void* stream) {
  if (stats) memset(stats, 0, sizeof(*stats));
  if (!c || !R || !sigma || !state || !offsets || !stats || rounds < 0 || rounds > 16) return CLSIMG_EINVAL;
  ST_TRY(check_geometry(a, g));
  ST_TRY(check_opts(o, a->P));
  if (o->nsamples <= 0 && o->kappa_d != 0.0) return CLSIMG_EINVAL;
  const int P = a->P, Q = g->nl * g->nm, Pp = pad_p(P), MT = Pp / 8;
  if (o->cost != CLSIMG_COST_LS || !beam_fits(P)) return CLSIMG_ENOTSUP;
  c->prec = o->precision;
  DeviceGuard guard(c->device);
  hipStream_t st = (hipStream_t)stream;
  ST_TRY(ensure_workspace(c, P, Q));
  ST_TRY(ensure(c, c->Flist, (size_t)Q * sizeof(int)));
  ST_TRY(ensure(c, c->Ulist, (size_t)Q * sizeof(int)));
  ST_TRY(ensure(c, c->x, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->lsqr2, 3 * sizeof(LsqrState)));
  ST_TRY(ensure(c, c->done, sizeof(int)));
  ST_TRY(ensure(c, c->bar, 2 * sizeof(unsigned)));
  ST_TRY(ensure(c, c->eps, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->mb_acc, (size_t)Q * sizeof(float)));  // on-grid bound gamma0
  ST_TRY(ensure(c, c->mb_acc2, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->xf, (size_t)Q * 2 * Pp * sizeof(float)));
  if (!mf_out) ST_TRY(ensure(c, c->mf, (size_t)Q * sizeof(float)));
  if (!gamma_out) ST_TRY(ensure(c, c->gamma, (size_t)Q * sizeof(float)));
  ST_TRY(ensure_tables(c, a, g, st));
  float* mf = mf_out ? mf_out : P_<float>(c->mf);
  float* gamma = gamma_out ? gamma_out : P_<float>(c->gamma);  // bounds in use (free pixels shifted)
  float* gamma0 = P_<float>(c->mb_acc);
  float* eps = P_<float>(c->eps);
  float* xf = P_<float>(c->xf);
  float* x = P_<float>(c->x);
  int* Flist = P_<int>(c->Flist);
  int* Ulist = P_<int>(c->Ulist);
  float2* B0 = P_<float2>(c->B0);
  float2* Bb = P_<float2>(c->Bb);
  float2* E = P_<float2>(c->E);
  uint64_t* keys = P_<uint64_t>(c->keys);
  SolveDecision* dec = P_<SolveDecision>(c->dec);
  LsqrState* S2 = P_<LsqrState>(c->lsqr2);
  LsqrState* Sfin = S2 + 2;
  int* done = P_<int>(c->done);
  unsigned* bar = P_<unsigned>(c->bar);
  int* lerr = reinterpret_cast<int*>(bar + 1);
  const int* grad_stop = &dec->grad_done;
  double* nrm = P_<double>(c->beta_part);
  const Tables tab = tables_of(c, g, P);
  const double* pos = P_<const double>(c->pos_d);
  const float2* Rf = reinterpret_cast<const float2*>(R);
  const float half_l = (float)(0.5 * fabs(g->dl)), half_m = (float)(0.5 * fabs(g->dm));
  // images, on-grid bound and threshold (Sec. II-D, App. A)
  const float eps_scale = o->kappa_d != 0.0 ? (float)(o->kappa_d / sqrt((double)o->nsamples)) : 0.f;
  ST_TRY(beam_full(c, g, P, Rf, BEAM_MF, mf, eps, eps_scale, 0, 0, 1.f, st));
  ST_TRY(compute_bound(c, R, a, g, o, gamma0, st));  // MVDR: leaves R^-1 in c->Rinv
  const int bkind = o->bound == CLSIMG_BOUND_MVDR ? 0 : (o->bound == CLSIMG_BOUND_MF ? 1 : 2);
  const double bkb = o->kappa_b == 0.0 ? 0.0
                     : (bkind == 0 ? o->kappa_b / sqrt((double)(o->nsamples - P - 1))
                                   : o->kappa_b / sqrt((double)o->nsamples));
  const float2* bmat = bkind == 0 ? P_<const float2>(c->Rinv) : Rf;
  HIP_TRY(hipMemcpyAsync(gamma, gamma0, (size_t)Q * sizeof(float), hipMemcpyDeviceToDevice, st));
  HIP_TRY(launch_sub_diag(Rf, noise_diag, P, B0, st));
  HIP_TRY(launch_frob2(B0, P * P, nrm, st));
  ST_TRY(read_back(c, c->h_norms, nrm, sizeof(double), st));
  const double b0norm = sqrt(c->h_norms[0]);
  HIP_TRY(launch_init_state(nullptr, nullptr, sigma, state, Q, st));
  HIP_TRY(launch_fill(offsets, 0.f, 2 * Q, st));
  auto xf_off = [&](int n) {
    return launch_xf_off(pos, P, a->lambda, g->nl, g->l0, g->dl, g->m0, g->dm, Flist, n, offsets, xf, st);
  };
  auto corr_xf = [&](int n, const float* vals, const int* gidx, const int* stop) {
    CorrOsParams cp;
    cp.MT = MT;
    cp.P = P;
    cp.xf = xf;
    cp.n = n;
    cp.vals = vals;
    cp.gidx = gidx;
    cp.out = E;
    cp.B = Bb;
    cp.cK = 1.f;
    cp.cB = -1.f;
    cp.frag = P_<float>(c->frag_r);
    cp.stop_flag = stop;
    return launch_corr_os(cp, st);
  };

  const int max_outer = o->max_outer < 0 ? 4 * Q : o->max_outer;
  int status = CLSIMG_OK;
  int outer = 0, adds = 0, drops = 0, lsqr_total = 0, itnlim_hits = 0, last_added = -1, nF = 0, nU = 0;
  bool need_solve = true;
  float lam_min = 0.f, eps_min = 0.f;
  int i_min = -1, st_min = 0;
  double margin_lambda = INFINITY, margin_z = INFINITY, flops = 2.0 * beam_flops(P, Q);
  for (;;) {
    if (need_solve) {
      if (outer >= max_outer) {
        status = CLSIMG_WMAXOUTER;
        break;
      }
      HIP_TRY(launch_compact(state, Q, Flist, Ulist, dec, st));
      HIP_TRY(launch_offgrid_sets(state, Q, gamma0, offsets, sigma, st));
      ST_TRY(read_back(c, c->h_dec, dec, sizeof(SolveDecision), st));
      nF = c->h_dec->nF;
      nU = c->h_dec->nU;
      if (nF > 0 && !lsqr_cu_fits(P, nF)) return CLSIMG_ENOTSUP;  // beyond the one-workgroup LSQR
      // b = B0 - Psi_U gamma0_U on the grid (eq. bsubproblemLS)
      ST_TRY(correlate(c, g, P, Ulist, gamma0, 1, nU, Bb, B0, -1.f, 1.f, nullptr, nullptr, nullptr, nullptr, st));
      flops += corr_flops(P, nU);
      const int itnlim = o->itnlim < 0 ? 4 * nF + 100 : o->itnlim;
      for (int t = 0; t <= rounds; ++t) {
        HIP_TRY(xf_off(nF));
        HIP_TRY(launch_lsqr_setup2(S2, done, bar, lerr, o->atol, o->btol, o->conlim, itnlim, st));
        if (nF > 0) {
          LsqrCuParams lc;
          lc.P = P;
          lc.n = nF;
          lc.xf = xf;
          lc.B = Bb;
          lc.x_out = x;
          lc.Sfinal = Sfin;
          lc.done = done;
          lc.atol = o->atol;
          lc.btol = o->btol;
          lc.conlim = o->conlim;
          lc.itnlim = itnlim;
          HIP_TRY(launch_lsqr_cu(lc, st));
        }
        if (t == rounds) break;
        ST_TRY(read_back(c, c->h_lsqr, Sfin, sizeof(LsqrState), st));
        lsqr_total += c->h_lsqr->itn;
        if (c->h_lsqr->istop == 7) ++itnlim_hits;
        flops += nF > 0 ? beam_flops(P, nF) + c->h_lsqr->itn * (corr_flops(P, nF) + beam_flops(P, nF)) : 0.0;
        // E = Psi(delta)_F z - b, then one Gauss-Newton step per free pixel
        HIP_TRY(corr_xf(nF, x, nullptr, nullptr));
        HIP_TRY(launch_newton_offset(E, P, pos, a->lambda, Flist, nF, x, xf, offsets, half_l, half_m, st));
      }
      // bounds of the free pixels at their shifted directions
      HIP_TRY(hipMemcpyAsync(gamma, gamma0, (size_t)Q * sizeof(float), hipMemcpyDeviceToDevice, st));
      HIP_TRY(launch_gamma_off(bkind, bmat, P, Flist, nF, xf, o->C, bkb, gamma, st));
      HIP_TRY(launch_step(done, lerr, Sfin, x, x, Flist, nF, sigma, gamma, state, dec, st));
      // gradient after a feasible subproblem: E = Psi(delta)_F sigma_F - b, multipliers on the grid
      HIP_TRY(corr_xf(nF, sigma, Flist, grad_stop));
      HIP_TRY(launch_beam_lambda(nullptr, E, P, tab, grad_stop, state, keys, nullptr, st));
      HIP_TRY(launch_argmin_final(keys, beam_grid(Q), eps, state, dec, st));
      ST_TRY(read_back(c, c->h_dec, dec, sizeof(SolveDecision), st));
      const SolveDecision d = *c->h_dec;
      if (nF > 0 && !d.lsqr_done) return CLSIMG_EHIP;  // the LSQR kernel did not finish
      ++outer;
      lsqr_total += d.lsqr_itn;
      if (nF > 0) flops += beam_flops(P, nF) + d.lsqr_itn * (corr_flops(P, nF) + beam_flops(P, nF));
      if (d.feasible) flops += corr_flops(P, nF) + beam_flops(P, Q);
      if (nF > 0 && d.lsqr_istop == 7) ++itnlim_hits;
      if (d.feasible) {
        need_solve = false;
        if (nF > 0) margin_z = std::min(margin_z, (double)d.margin_z);
        if (d.i_min < 0) break;
        lam_min = d.lam_min;
        eps_min = d.eps_min;
        i_min = d.i_min;
        st_min = d.st_min;
      } else {
        ++drops;
        need_solve = true;
        if (d.ib == last_added && d.mu_max == 0.0f) {
          status = CLSIMG_WCYCLE;
          break;
        }
      }
      last_added = -1;
    } else {
      if (eps_min > 0.f) margin_lambda = std::min(margin_lambda, fabs((double)lam_min + eps_min) / eps_min);
      if (lam_min < -eps_min) {
        HIP_TRY(launch_set_state(state, i_min, (uint8_t)CLSIMG_STATE_F, st));
        ++adds;
        last_added = i_min;
        need_solve = true;
      } else {
        break;
      }
    }
  }
  if (status == CLSIMG_OK && itnlim_hits) status = CLSIMG_WITNLIM;
  // final sets, upper-set powers and offsets; residual ||B0 - Psi_U gamma0_U - Psi(delta)_F sigma_F||
  HIP_TRY(launch_compact(state, Q, Flist, Ulist, dec, st));
  HIP_TRY(launch_offgrid_sets(state, Q, gamma0, offsets, sigma, st));
  ST_TRY(read_back(c, c->h_dec, dec, sizeof(SolveDecision), st));
  nF = c->h_dec->nF;
  nU = c->h_dec->nU;
  ST_TRY(correlate(c, g, P, Ulist, gamma0, 1, nU, Bb, B0, -1.f, 1.f, nullptr, nullptr, nullptr, nullptr, st));
  HIP_TRY(xf_off(nF));
  HIP_TRY(corr_xf(nF, sigma, Flist, nullptr));
  HIP_TRY(launch_frob2(E, P * P, nrm, st));
  ST_TRY(read_back(c, c->h_norms, nrm, sizeof(double), st));
  const double rn = sqrt(c->h_norms[0]);
  stats->status = status;
  stats->outer_iters = outer;
  stats->adds = adds;
  stats->drops = drops;
  stats->lsqr_iters_total = lsqr_total;
  stats->lsqr_itnlim_hits = itnlim_hits;
  stats->nF = nF;
  stats->nU = nU;
  stats->rel_residual = b0norm > 0 ? rn / b0norm : 0.0;
  stats->objective = 0.5 * rn * rn;
  stats->min_margin_lambda = margin_lambda;
  stats->min_margin_z = margin_z;
  stats->psi_flops = flops;
  return status;
}

int clsimg_solve_batch(clsimg_ctx* c, int32_t n, clsimg_request* reqs, const clsimg_opts* o, void* stream) {
  if (!c || !reqs || n < 1) return CLSIMG_EINVAL;
  for (int r = 0; r < n; ++r) memset(&reqs[r].stats, 0, sizeof(clsimg_stats));
  const int P = reqs[0].array.P;
  ST_TRY(check_opts(o, P));
  if (o->nsamples <= 0 && o->kappa_d != 0.0) return CLSIMG_EINVAL;
  const bool pwls = o->cost == CLSIMG_COST_PWLS;
  if (pwls && o->nsamples <= P + 1 && o->kappa_d != 0.0) return CLSIMG_EINVAL;
  int Qmax = 0, nlmax = 0, nmmax = 0;
  for (int r = 0; r < n; ++r) {
    const clsimg_request& q = reqs[r];
    if (!q.R || !q.sigma || !q.state || q.array.P != P) return CLSIMG_EINVAL;
    ST_TRY(check_geometry(&q.array, &q.grid));
    Qmax = std::max(Qmax, q.grid.nl * q.grid.nm);
    nlmax = std::max(nlmax, q.grid.nl);
    nmmax = std::max(nmmax, q.grid.nm);
  }
  if (!request_on_device(P)) return CLSIMG_ENOTSUP;
  DeviceGuard guard(c->device);
  hipStream_t st = (hipStream_t)stream;
  ST_TRY(ensure_workspace(c, P, Qmax));
  ST_TRY(ensure(c, c->eps, (size_t)Qmax * sizeof(float)));
  if (pwls) ST_TRY(ensure(c, c->pw_h, (size_t)Qmax * sizeof(float)));

  // per-request slices of one workspace, all laid out for the largest grid
  const int tiles = beam_batch_tiles(n, Qmax);
  const int bpr = beam_grid_batched(Qmax, tiles);  // multiplier blocks per request in the launch
  ReqLayout L = request_layout(P, nlmax, nmmax, pwls, bpr);
  L.tiles = tiles;
  ST_TRY(ensure(c, c->batch, L.bytes * n));
  // the least-squares cost with the MVDR bound (factored below), FP32: the
  // per-request set-up launches become two batched launches
  const bool fused = !pwls && o->bound == CLSIMG_BOUND_MVDR && P <= kCholLdsMaxP &&
                     o->precision == CLSIMG_FP32 && !c->beam_prep;
  bool shared_tables = fused;
  for (int r = 1; r < n && shared_tables; ++r) {
    const clsimg_array &a0 = reqs[0].array, &a = reqs[r].array;
    shared_tables = a.lambda == a0.lambda && memcmp(&reqs[r].grid, &reqs[0].grid, sizeof(clsimg_grid)) == 0 &&
                    memcmp(a.pos_xy, a0.pos_xy, sizeof(double) * 2 * P) == 0;
  }
  // device parameters: outer-step parameters and multiplier items (then the
  // set-up items), then the gathered outer states, the factorisation items
  // and their statuses
  const bool own_tables = fused && !shared_tables;
  const size_t pbytes =
      (size_t)n * (sizeof(OuterParams) + sizeof(BeamLamItem) +
                   (fused ? sizeof(ReqInitItem) + sizeof(BeamSetItem) : 0) +
                   (own_tables ? sizeof(TableItem) + sizeof(double) * 2 * P : 0));
  const size_t off_st = (pbytes + 255) & ~(size_t)255;
  const size_t off_ci = (off_st + (size_t)n * sizeof(OuterState) + 255) & ~(size_t)255;
  const size_t off_cs = (off_ci + (size_t)n * sizeof(CholItem) + 255) & ~(size_t)255;
  ST_TRY(ensure(c, c->batch_params, off_cs + (size_t)n * sizeof(int)));
  const size_t hbytes = std::max({pbytes, (size_t)n * sizeof(OuterState), (size_t)n * sizeof(CholItem)});
  if (c->h_batch_bytes < hbytes) {
    if (c->h_batch) {
      HIP_TRY(hipStreamSynchronize(st));
      (void)hipHostFree(c->h_batch);
      c->h_batch = nullptr;
      c->h_batch_bytes = 0;
    }
    HIP_TRY(hipHostMalloc((void**)&c->h_batch, hbytes, hipHostMallocDefault));
    c->h_batch_bytes = hbytes;
  } else {
    HIP_TRY(hipStreamSynchronize(st));  // the staging of a previous call has been consumed
  }
  char* base = P_<char>(c->batch);
  auto slice = [&](int r) { return base + (size_t)r * L.bytes; };
  char* dbase = P_<char>(c->batch_params);
  // MVDR bound of the least-squares cost: every request's R^-1 from one
  // factorisation launch (one workgroup each), checked with one read-back
  const float2* rinv = nullptr;
  if (!pwls && o->bound == CLSIMG_BOUND_MVDR && P <= kCholLdsMaxP) {
    ST_TRY(ensure(c, c->batch_rinv, (size_t)n * P * P * sizeof(float2)));
    CholItem* hc = reinterpret_cast<CholItem*>(c->h_batch);
    int* dstat = reinterpret_cast<int*>(dbase + off_cs);
    for (int r = 0; r < n; ++r)
      hc[r] = CholItem{reinterpret_cast<const float2*>(reqs[r].R), nullptr,
                       P_<float2>(c->batch_rinv) + (size_t)r * P * P, dstat + r};
    CholItem* dc = reinterpret_cast<CholItem*>(dbase + off_ci);
    HIP_TRY(hipMemcpyAsync(dc, hc, (size_t)n * sizeof(CholItem), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_chol_inverse_batch(dc, n, P, st));
    int* hstat = reinterpret_cast<int*>(c->h_batch);  // the items' upload is done once this copy is
    ST_TRY(read_back(c, hstat, dstat, (size_t)n * sizeof(int), st));
    for (int r = 0; r < n; ++r)
      if (hstat[r] != 0) return CLSIMG_ENOTPD;
    rinv = P_<const float2>(c->batch_rinv);
  }
  const size_t off_ii = (size_t)n * (sizeof(OuterParams) + sizeof(BeamLamItem));
  const size_t off_bi = off_ii + (size_t)n * sizeof(ReqInitItem);
  const size_t off_ti = off_bi + (size_t)n * sizeof(BeamSetItem);
  const size_t off_pos = off_ti + (size_t)n * sizeof(TableItem);
  OuterParams* hp = reinterpret_cast<OuterParams*>(c->h_batch);
  BeamLamItem* hi = reinterpret_cast<BeamLamItem*>(c->h_batch + (size_t)n * sizeof(OuterParams));
  for (int r = 0; r < n; ++r) {
    SetupItems items{reinterpret_cast<ReqInitItem*>(c->h_batch + off_ii) + r,
                     reinterpret_cast<BeamSetItem*>(c->h_batch + off_bi) + r,
                     shared_tables,
                     own_tables ? reinterpret_cast<TableItem*>(c->h_batch + off_ti) + r : nullptr,
                     own_tables ? reinterpret_cast<double*>(c->h_batch + off_pos) + (size_t)r * 2 * P : nullptr,
                     own_tables ? reinterpret_cast<const double*>(dbase + off_pos) + (size_t)r * 2 * P : nullptr};
    ST_TRY(request_setup(c, reqs[r], o, slice(r), L, hp[r], hi[r], st, rinv ? rinv + (size_t)r * P * P : nullptr,
                         fused && rinv ? &items : nullptr));
  }
  OuterParams* dp = P_<OuterParams>(c->batch_params);
  BeamLamItem* di = reinterpret_cast<BeamLamItem*>(P_<char>(c->batch_params) + (size_t)n * sizeof(OuterParams));
  HIP_TRY(hipMemcpyAsync(dp, c->h_batch, pbytes, hipMemcpyHostToDevice, st));
  if (fused && rinv) {
    if (own_tables)
      HIP_TRY(launch_tables_batch(reinterpret_cast<const TableItem*>(dbase + off_ti), n, pad_p(P) * (nlmax + nmmax),
                                  st));
    HIP_TRY(launch_request_init_batch(reinterpret_cast<const ReqInitItem*>(dbase + off_ii), n, Qmax, st));
    HIP_TRY(launch_beam_setup_batch(reinterpret_cast<const BeamSetItem*>(dbase + off_bi), n, bpr, P, st));
  }
  // wait for the upload before the staging is reused for the state read-backs
  HIP_TRY(hipStreamSynchronize(st));

  int nb = 8;
  for (;;) {
    for (int b = 0; b < nb; ++b) {
      HIP_TRY(launch_outer_step_batch(dp, n, P, st));
      HIP_TRY(launch_beam_lambda_batch(di, n, bpr, P, st));
    }
    OuterState* hs = reinterpret_cast<OuterState*>(c->h_batch);
    OuterState* ds = reinterpret_cast<OuterState*>(dbase + off_st);
    HIP_TRY(launch_gather_states(dp, n, ds, st));
    HIP_TRY(hipMemcpyAsync(hs, ds, (size_t)n * sizeof(OuterState), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    bool all = true;
    for (int r = 0; r < n; ++r) all = all && hs[r].done;
    if (all) break;
    nb = std::min(2 * nb, 128);
  }
  const OuterState* hs = reinterpret_cast<const OuterState*>(c->h_batch);
  int worst = CLSIMG_OK;
  for (int r = 0; r < n; ++r) {
    const int status = request_finish(reqs[r], o, slice(r), L, hs[r], st);
    if (status < 0) worst = (worst < 0) ? worst : status;
    else if (worst >= 0 && status > worst) worst = status;
  }
  return worst;
}

}  // extern "C"
