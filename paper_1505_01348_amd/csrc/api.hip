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
#include "workspace.h"

using namespace clsimg;

namespace {

// refined multipliers: at most Q / 8 (64 .. this many) FP32 candidates per
// step (else the step's multipliers are all evaluated in FP32), and the |W|
// partial count
constexpr int kCandCap = 16384;
constexpr int kCandAbsParts = 256;

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
  DevBuf El, Em, ElT, EmT, pos_d;
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
  DevBuf pw_T, pw_Bw, pw_Eh, pw_nrm;  // PWLS on the host-driven loop: products with L^-1, whitened b and E
  DevBuf cpart;                       // per-chunk counts of the compaction
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
  bool coop = false;   // cooperative launches available (multi-workgroup LSQR kernel)
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
  void* scratch = nullptr;    // this device's copy of the static workspace (allocation-free calls)
  // device time of the host-driven loop's multiplier kernel (clsimg_kernel_timing)
  bool time_mult = false;
  hipEvent_t tm_ev[2] = {nullptr, nullptr};
  double tm_ms = 0.0;
  int tm_n = 0;
  // captured round of batched Table I steps (clsimg_opts.batch_graph): its
  // launch arguments, the capture stream and the executable graph
  hipStream_t cap_st = nullptr;
  hipGraphExec_t round_exec = nullptr;
  const void* round_key[2] = {nullptr, nullptr};
  int round_key_n = 0, round_key_bpr = 0, round_key_P = 0;
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
  ST_TRY(ensure(c, c->ElT, (size_t)corr_rows(Pp) * g->nl * sizeof(float2)));
  ST_TRY(ensure(c, c->EmT, (size_t)corr_rows(Pp) * g->nm * sizeof(float2)));
  HIP_TRY(launch_tables_t(P_<const float2>(c->El), P_<const float2>(c->Em), Pp, g->nl, g->nm, P_<float2>(c->ElT),
                          P_<float2>(c->EmT), st));
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
  // the antenna-fastest copies belong to the context's own tables
  const bool own = !c->tab_El && !c->tab_Em;
  t.ElT = own ? P_<const float2>(c->ElT) : nullptr;
  t.EmT = own ? P_<const float2>(c->EmT) : nullptr;
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
  ST_TRY(ensure(c, c->W, chol_work_elems(P) * sizeof(double2)));  // Cholesky beyond 64 antennas
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
  const bool small = corr_small_fits(n, 1);  // a short list: one launch straight into the output
  if (!small && (size_t)nchunks * forward_part_floats(P) > c->part.bytes / sizeof(float)) return CLSIMG_EINVAL;
  FwdParams f;
  if (n > 0) {
    f.tab = tables_of(c, g, P);
    f.MT = MT;
    f.idx = idx;
    f.vals = vals;
    f.gather = gather;
    f.n = n;
    f.chw = chw;
    f.part = P_<float>(c->part);
    f.stop_flag = stop;
    if (!small) HIP_TRY(launch_forward(f, st));
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
  if (small) HIP_TRY(launch_corr_small(f, r, st));
  else HIP_TRY(launch_reduce(r, st));
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
    ST_TRY(ensure(c, c->hscale, kHalfScaleFloats * sizeof(float)));
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
  // fragments built inside the kernel
  const float* fb = nullptr;
  const float2* Uk = U;
  switch (kind) {
    case BEAM_MF: HIP_TRY(launch_beam_mf(fb, Uk, P, tab, out, eps, eps_scale, st, ts)); break;
    case BEAM_MVDR: HIP_TRY(launch_beam_mvdr(fb, Uk, P, tab, out, C, kb, st)); break;
    default: HIP_TRY(launch_beam_store(fb, Uk, P, tab, out, scale, st)); break;
  }
  return CLSIMG_OK;
}

// A small device-to-host read in stream order (pinned host memory): the copy,
// then an event polled until it completes.  The host usually reaches the wait
// long before the GPU reaches the copy; polling keeps the wake-up to a few
// microseconds, where a blocking stream synchronisation would sleep and be
// woken late.  One event per host thread and device, created on first use.
int read_back(clsimg_ctx* c, void* host, const void* dev, size_t bytes, hipStream_t st) {
  (void)c;
  thread_local int ev_dev = -1;
  thread_local hipEvent_t ev = nullptr;
  int d = 0;
  HIP_TRY(hipGetDevice(&d));
  if (d != ev_dev) {
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ev = e;  // an event of another device is kept (one per thread and device switch)
    ev_dev = d;
  }
  HIP_TRY(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(ev, st));
  for (;;) {
    const hipError_t e = hipEventQuery(ev);
    if (e == hipSuccess) break;
    if (e != hipErrorNotReady) return CLSIMG_EHIP;
  }
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
  if (o->loop != CLSIMG_LOOP_AUTO && o->loop != CLSIMG_LOOP_HOST) return CLSIMG_EINVAL;
  if (o->lsqr_engine < CLSIMG_LSQR_AUTO || o->lsqr_engine > CLSIMG_LSQR_TWO_KERNEL) return CLSIMG_EINVAL;
  if (o->hand_over_free < 0 || (o->trace != 0 && o->trace != 1)) return CLSIMG_EINVAL;
  if (o->batch_graph != 0 && o->batch_graph != 1) return CLSIMG_EINVAL;
  return CLSIMG_OK;
}

// largest free set a device-resident loop keeps before continuing on the host
int hand_over_limit(const clsimg_opts* o) { return o->hand_over_free > 0 ? o->hand_over_free : (1 << 30); }

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
    if (pwls || !rinv || o->bound != CLSIMG_BOUND_MVDR || c->prec != CLSIMG_FP32 || !beam_fits(P))
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
  op.max_f = hand_over_limit(o);
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
  o->loop = CLSIMG_LOOP_AUTO;
  o->lsqr_engine = CLSIMG_LSQR_AUTO;
  o->hand_over_free = 0;
  o->trace = 0;
  o->batch_graph = 0;
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
  int coop = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) == hipSuccess)
    c->coop = coop != 0;
  void* hp = nullptr;
  // room for the norm partials of the largest array (reduce_blocks grows as P^2), or one per row
  const int nnorm = std::max(reduce_blocks(CLSIMG_MAX_P), CLSIMG_MAX_P);
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
  DevBuf* bufs[] = {&c->El,   &c->Em,    &c->ElT, &c->EmT, &c->pos_d,    &c->frag_r, &c->frag_u, &c->frag_b, &c->ostate, &c->pw_h, &c->pw_rs, &c->pw_g, &c->pw_eps, &c->pw_dinv, &c->pw_Lw, &c->pw_B0w, &c->pw_T, &c->pw_Bw, &c->pw_Eh, &c->pw_nrm, &c->cpart, &c->batch, &c->batch_params, &c->batch_rinv, &c->part,  &c->beta_part,
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
  if (c->round_exec) (void)hipGraphExecDestroy(c->round_exec);
  if (c->cap_st) (void)hipStreamDestroy(c->cap_st);
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
    case CLSIMG_EWORKSPACE: return "device workspace missing or too small (internal check)";
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
  const size_t o_fr = take(fb), o_sc = take(kHalfScaleFloats * sizeof(float));
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

namespace {

// The sets' index lists F and U and their sizes (dec->nF, dec->nU), after
// checking that the lists and the decision record exist at the sizes the
// compaction writes.
int compact(clsimg_ctx* c, const uint8_t* state, int Q, hipStream_t st) {
  const size_t np = (size_t)compact_parts(Q) * sizeof(int);
  if (c->cpart.bytes < np) ST_TRY(ensure(c, c->cpart, np));
  ST_TRY(need_all({{&c->Flist, (size_t)Q * sizeof(int)}, {&c->Ulist, (size_t)Q * sizeof(int)},
                   {&c->dec, sizeof(SolveDecision)}, {&c->cpart, np}}));
  HIP_TRY(launch_compact(state, Q, P_<int>(c->Flist), P_<int>(c->Ulist), P_<SolveDecision>(c->dec),
                         P_<int>(c->cpart), st));
  return CLSIMG_OK;
}

// What the phases of clsimg_solve share: set-up (images, bound, data, the
// starting sets), the device-resident loop (Table I on the device), the
// host-driven loop (one subproblem per round trip) and the statistics.
struct SolveRun {
  clsimg_ctx* c = nullptr;
  const clsimg_grid* g = nullptr;
  const clsimg_opts* o = nullptr;
  hipStream_t st = nullptr;
  int P = 0, Q = 0, MT = 0, nbeta = 0, nfw = 0, ntiles_Q = 0, max_outer = 0, cand_cap = 0, cand_tile = 0;
  bool pwls = false, device_loop = false, fused = false, beam_half = false, beam_full_grid = false,
       beam_big_grid_ok = false;
  // device buffers
  float *sigma = nullptr, *mf = nullptr, *gamma = nullptr, *eps = nullptr;
  uint8_t* state = nullptr;
  float2 *B0 = nullptr, *Bb = nullptr, *u = nullptr, *E = nullptr;
  int *Flist = nullptr, *Ulist = nullptr, *done = nullptr, *lerr = nullptr;
  float *v = nullptr, *w = nullptr, *x = nullptr, *x1 = nullptr, *w1 = nullptr, *vraw = nullptr, *xf = nullptr;
  float *frag_r = nullptr, *frag_u = nullptr;
  double *beta_part = nullptr, *alpha_part = nullptr, *bparts[2] = {nullptr, nullptr};
  uint64_t* keys = nullptr;
  LsqrState *ls = nullptr, *S2 = nullptr, *Sfin = nullptr;
  SolveDecision* dec = nullptr;
  unsigned* bar = nullptr;
  const int* lsqr_stop = nullptr;
  const int* grad_stop = nullptr;
  // PWLS operands (eq. preWLS), else the LS ones
  const float* lam_scale = nullptr;
  const float* op_gamma = nullptr;
  const float* op_eps = nullptr;
  const float2* op_B0 = nullptr;
  Stamps mult_stamps;
  // iteration state
  int status = CLSIMG_OK, outer = 0, adds = 0, drops = 0, lsqr_total = 0, itnlim_hits = 0, last_added = -1;
  int nF = 0, nU = 0, batch = 4, i_min = -1, st_min = 0;
  bool need_solve = true, host_loop = true, stop = false;
  float lam_min = 0.f, eps_min = 0.f;
  double margin_lambda = INFINITY, margin_z = INFINITY;
  double flops = 0.0, b0norm = 0.0, dev_res2 = 0.0, dev_b0n2 = 0.0;

  Tables tab() const { return tables_of(c, g, P); }
  AdjParams lsqr_adj(const int* stop_flag) const {
    AdjParams a = adj_params(c, g, P, frag_u, Flist, nF, stop_flag);
    a.xf = xf;
    return a;
  }
  // the LSQR adjoint of the split-K engine: for large arrays its rows are
  // split over workgroups, with the correlation's partial buffer (free by
  // then) as the workspace of the row groups' dots
  AdjParams lsqr_adj_rows(const int* stop_flag) const {
    AdjParams a = adj_params(c, g, P, frag_u, Flist, nF, stop_flag);
    a.rows_part = P_<float>(c->part);
    a.rows_cap = c->part.bytes / sizeof(float);
    return a;
  }
  LsqrFwdParams fwd_params(int iter, int nalpha2) const {
    LsqrFwdParams f;
    f.tab = tab();
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
  }
};

// Workspace, images, bound and threshold (Sec. II-D, App. A), the data B0 =
// R - diag(noise), the starting image and sets; the PWLS inputs.
int solve_setup(SolveRun& r, const clsimg_c32* R, const clsimg_array* a, const float* noise_diag,
                const float* sigma0, const uint8_t* state0, float* mf_out, float* gamma_out) {
  clsimg_ctx* c = r.c;
  const clsimg_opts* o = r.o;
  hipStream_t st = r.st;
  const int P = r.P, Q = r.Q;
  ST_TRY(ensure_workspace(c, P, Q));
  ST_TRY(ensure(c, c->Flist, (size_t)Q * sizeof(int)));
  ST_TRY(ensure(c, c->Ulist, (size_t)2 * Q * sizeof(int)));  // two buffers for the device loop
  ST_TRY(ensure(c, c->ostate, sizeof(OuterState)));
  for (DevBuf* b : {&c->v, &c->w, &c->x, &c->x1, &c->w1, &c->vraw}) ST_TRY(ensure(c, *b, (size_t)Q * sizeof(float)));
  ST_TRY(ensure(c, c->lsqr2, 3 * sizeof(LsqrState)));
  ST_TRY(ensure(c, c->done, sizeof(int)));
  ST_TRY(ensure(c, c->bar, 2 * sizeof(unsigned)));
  const int nparts = std::max(std::max(reduce_blocks(P), lsqr_fwd_waves(P)), Q / 32 + 64);
  ST_TRY(ensure(c, c->bpart0, (size_t)nparts * sizeof(double)));
  ST_TRY(ensure(c, c->bpart1, (size_t)nparts * sizeof(double)));
  const size_t nalpha_max = (size_t)(Q / 16 + 64);  // one per 16-pixel tile
  ST_TRY(ensure(c, c->alpha_part, nalpha_max * sizeof(double)));

  // PWLS: on the device-resident loop, or on the host-driven loop with the
  // whitened steering rows in the free-set cache (up to 12 row tiles, P <= 96)
  r.pwls = o->cost == CLSIMG_COST_PWLS;
  r.device_loop = beam_fits(P) && outer_fits(P) && o->loop == CLSIMG_LOOP_AUTO && !o->trace;
  if (r.pwls && pad_p(P) / 8 > 12) return CLSIMG_ENOTSUP;
  if (r.pwls && o->nsamples <= P + 1 && o->kappa_d != 0.0) return CLSIMG_EINVAL;
  if (r.pwls) {
    for (DevBuf* b : {&c->pw_h, &c->pw_rs, &c->pw_g, &c->pw_eps, &c->pw_dinv})
      ST_TRY(ensure(c, *b, (size_t)Q * sizeof(float)));
    ST_TRY(ensure(c, c->pw_Lw, (size_t)P * P * sizeof(float2)));
    ST_TRY(ensure(c, c->pw_B0w, (size_t)P * P * sizeof(float2)));
    ST_TRY(ensure(c, c->pw_T, (size_t)P * P * sizeof(double2)));
    ST_TRY(ensure(c, c->pw_Bw, (size_t)P * P * sizeof(float2)));
    ST_TRY(ensure(c, c->pw_Eh, (size_t)P * P * sizeof(float2)));
    ST_TRY(ensure(c, c->pw_nrm, (size_t)P * sizeof(double)));
  }
  ST_TRY(ensure(c, c->eps, (size_t)Q * sizeof(float)));
  if (!mf_out) ST_TRY(ensure(c, c->mf, (size_t)Q * sizeof(float)));
  if (!gamma_out) ST_TRY(ensure(c, c->gamma, (size_t)Q * sizeof(float)));
  ST_TRY(ensure_tables(c, a, r.g, st));

  r.MT = pad_p(P) / 8;
  r.fused = r.MT <= 12;  // the two-kernel LSQR step and its free-set cache up to 12 row tiles (P <= 96)
  r.nbeta = reduce_blocks(P);
  r.nfw = lsqr_fwd_waves(P);
  r.ntiles_Q = ntiles_adj(P, Q);
  r.max_outer = o->max_outer < 0 ? 4 * Q : o->max_outer;
  r.beam_full_grid = beam_fits(P);
  r.beam_big_grid_ok = !beam_fits(P) && beam_big_fits(P);
  // timing of the multiplier kernel (clsimg_kernel_timing): events bound to its launches
  r.mult_stamps = c->time_mult ? Stamps{c->tm_ev[0], c->tm_ev[1]} : Stamps{};
  // reduced precision: the multipliers from one half-precision product, the
  // decision refined in FP32 over the candidates the rounding bound leaves
  r.beam_half = c->prec != CLSIMG_FP32;
  r.cand_cap = std::max(64, std::min(Q / 8, kCandCap));
  r.cand_tile = adjoint_tile_width(r.MT);
  if (r.beam_half) {
    ST_TRY(ensure(c, c->frag_h, std::max(beam_h16_frag_bytes(P), beam_h1_frag_bytes(P))));
    ST_TRY(ensure(c, c->hscale, kHalfScaleFloats * sizeof(float)));
    ST_TRY(ensure(c, c->mx_abs, kCandAbsParts * sizeof(double)));
    ST_TRY(ensure(c, c->mx_lam, (size_t)Q * sizeof(float)));
    ST_TRY(ensure(c, c->mx_cand, (size_t)r.cand_cap * sizeof(int)));
    ST_TRY(ensure(c, c->mx_count, sizeof(int)));
    const size_t nk = (size_t)std::max(beam_big_grid(P, Q, 2), (r.cand_cap + r.cand_tile - 1) / r.cand_tile) + 1;
    if (c->keys.bytes < nk * sizeof(uint64_t)) ST_TRY(ensure(c, c->keys, nk * sizeof(uint64_t)));
    const size_t rows = (size_t)((r.MT + 3) / 4) * 8 * r.cand_cap;  // row groups x K slices x list
    if (c->part.bytes < rows * sizeof(float)) ST_TRY(ensure(c, c->part, rows * sizeof(float)));
  }
  // every buffer the phases launch with, at the sizes their kernels assume
  const size_t fq = (size_t)Q * sizeof(float), cx = (size_t)P * P * sizeof(float2);
  ST_TRY(need_all({{&c->B0, cx},
                   {&c->Bb, cx},
                   {&c->u, cx},
                   {&c->E, cx},
                   {&c->Flist, (size_t)Q * sizeof(int)},
                   {&c->Ulist, (size_t)2 * Q * sizeof(int)},
                   {&c->v, fq},
                   {&c->w, fq},
                   {&c->x, fq},
                   {&c->x1, fq},
                   {&c->w1, fq},
                   {&c->vraw, fq},
                   {&c->eps, fq},
                   {&c->frag_r, (size_t)4 * pad_p(P) * pad_p(P) * sizeof(float)},
                   {&c->frag_u, (size_t)4 * pad_p(P) * pad_p(P) * sizeof(float)},
                   {&c->beta_part, (size_t)r.nbeta * sizeof(double)},
                   {&c->alpha_part, nalpha_max * sizeof(double)},
                   {&c->bpart0, (size_t)nparts * sizeof(double)},
                   {&c->bpart1, (size_t)nparts * sizeof(double)},
                   {&c->keys, (size_t)(std::max(r.ntiles_Q, beam_grid(Q)) + 1) * sizeof(uint64_t)},
                   {&c->lsqr, sizeof(LsqrState)},
                   {&c->lsqr2, 3 * sizeof(LsqrState)},
                   {&c->dec, sizeof(SolveDecision)},
                   {&c->done, sizeof(int)},
                   {&c->bar, 2 * sizeof(unsigned)},
                   {&c->ostate, sizeof(OuterState)}}));
  if (!mf_out) ST_TRY(need_all({{&c->mf, fq}}));
  if (!gamma_out) ST_TRY(need_all({{&c->gamma, fq}}));
  if (r.beam_half)
    ST_TRY(need_all({{&c->mx_lam, fq}, {&c->mx_cand, (size_t)r.cand_cap * sizeof(int)}, {&c->mx_count, sizeof(int)},
                     {&c->mx_abs, kCandAbsParts * sizeof(double)}, {&c->hscale, kHalfScaleFloats * sizeof(float)}}));
  if (r.pwls)
    ST_TRY(need_all({{&c->pw_h, fq}, {&c->pw_rs, fq}, {&c->pw_g, fq}, {&c->pw_eps, fq}, {&c->pw_dinv, fq},
                     {&c->pw_Lw, cx}, {&c->pw_B0w, cx}, {&c->pw_T, (size_t)P * P * sizeof(double2)},
                     {&c->pw_Bw, cx}, {&c->pw_Eh, cx}, {&c->pw_nrm, (size_t)P * sizeof(double)},
                     {&c->Li, (size_t)P * P * sizeof(double2)}}));

  r.mf = mf_out ? mf_out : P_<float>(c->mf);
  r.gamma = gamma_out ? gamma_out : P_<float>(c->gamma);
  r.eps = P_<float>(c->eps);
  r.B0 = P_<float2>(c->B0);
  r.Bb = P_<float2>(c->Bb);
  r.u = P_<float2>(c->u);
  r.E = P_<float2>(c->E);
  r.Flist = P_<int>(c->Flist);
  r.Ulist = P_<int>(c->Ulist);
  r.v = P_<float>(c->v);
  r.w = P_<float>(c->w);
  r.x = P_<float>(c->x);
  r.x1 = P_<float>(c->x1);
  r.w1 = P_<float>(c->w1);
  r.vraw = P_<float>(c->vraw);
  r.xf = P_<float>(c->xf);
  r.frag_r = P_<float>(c->frag_r);
  r.frag_u = P_<float>(c->frag_u);
  r.beta_part = P_<double>(c->beta_part);
  r.alpha_part = P_<double>(c->alpha_part);
  r.bparts[0] = P_<double>(c->bpart0);
  r.bparts[1] = P_<double>(c->bpart1);
  r.keys = P_<uint64_t>(c->keys);
  r.ls = P_<LsqrState>(c->lsqr);
  r.S2 = P_<LsqrState>(c->lsqr2);
  r.Sfin = r.S2 + 2;
  r.dec = P_<SolveDecision>(c->dec);
  r.done = P_<int>(c->done);
  r.bar = P_<unsigned>(c->bar);
  r.lerr = reinterpret_cast<int*>(r.bar + 1);
  r.lsqr_stop = &r.ls->done;
  r.grad_stop = &r.dec->grad_done;

  const float2* Rf = reinterpret_cast<const float2*>(R);
  r.flops = beam_flops(P, Q) + (o->bound != CLSIMG_BOUND_NONE ? beam_flops(P, Q) : 0.0);
  // bounds and threshold (Sec. II-D, App. A)
  const float eps_scale = o->kappa_d != 0.0 ? (float)(o->kappa_d / sqrt((double)o->nsamples)) : 0.f;
  if (beam_any(P)) {
    ST_TRY(beam_full(c, r.g, P, Rf, BEAM_MF, r.mf, r.eps, eps_scale, 0, 0, 1.f, st));
  } else {
    HIP_TRY(launch_adjoint_mf(adj_params(c, r.g, P, nullptr, nullptr, Q, nullptr, Rf), r.mf, r.eps, eps_scale,
                              st));
  }
  ST_TRY(compute_bound(c, R, a, r.g, o, r.gamma, st));
  // data B0 = R - diag(noise), its norm, the starting image and sets
  HIP_TRY(launch_sub_diag(Rf, noise_diag, P, r.B0, st));
  ST_TRY(correlate(c, r.g, P, nullptr, nullptr, 0, 0, r.E, r.B0, 0.f, 1.f, nullptr, nullptr, r.beta_part, nullptr,
                   st));
  HIP_TRY(hipMemcpyAsync(c->h_norms, r.beta_part, r.nbeta * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(launch_init_state(sigma0, state0, r.sigma, r.state, Q, st));
  ST_TRY(compact(c, r.state, Q, st));
  ST_TRY(read_back(c, c->h_dec, r.dec, sizeof(SolveDecision), st));
  r.b0norm = sqrt(sum_host(c->h_norms, r.nbeta));
  r.nF = c->h_dec->nF;
  r.nU = c->h_dec->nU;

  // PWLS inputs (eq. preWLS): Cholesky of R, h = a^H R^-1 a, D = h^2 / C, the
  // whitened data, bound D gamma and the MVDR-image threshold; the loop then
  // solves for D sigma
  r.op_gamma = r.gamma;
  r.op_eps = r.eps;
  r.op_B0 = r.B0;
  if (r.pwls) {
    if (o->bound != CLSIMG_BOUND_MVDR) {  // the MVDR bound has factorised R already
      HIP_TRY(launch_chol_inverse(Rf, P, P_<double2>(c->W), P_<double2>(c->Li), P_<float2>(c->Rinv),
                                  P_<int>(c->status), st));
      ST_TRY(read_back(c, c->h_status, c->status.ptr, sizeof(int), st));
      if (*c->h_status != 0) return CLSIMG_ENOTPD;
    }
    float* h = P_<float>(c->pw_h);
    ST_TRY(beam_full(c, r.g, P, P_<const float2>(c->Rinv), BEAM_STORE, h, nullptr, 0.f, 0, 0, 1.f, st));
    const double kd = o->kappa_d != 0.0 ? o->kappa_d / sqrt((double)(o->nsamples - P - 1)) : 0.0;
    HIP_TRY(launch_pwls_setup(h, r.gamma, o->C, kd, Q, P_<float>(c->pw_rs), P_<float>(c->pw_g),
                              P_<float>(c->pw_eps), P_<float>(c->pw_dinv), st));
    const double2* Li = P_<const double2>(c->Li);
    if (P <= 48) {  // L^-1 in FP32 for the device loop, and the whitened data
      HIP_TRY(launch_pwls_whiten(Li, r.B0, P, P_<float2>(c->pw_Lw), P_<float2>(c->pw_B0w), st));
      HIP_TRY(launch_pwls_sandwich(Li, r.B0, P, false, P_<double2>(c->pw_T), P_<float2>(c->pw_Bw),
                                   P_<double>(c->pw_nrm), st));  // its norm only
    } else {
      HIP_TRY(launch_pwls_sandwich(Li, r.B0, P, false, P_<double2>(c->pw_T), P_<float2>(c->pw_B0w),
                                   P_<double>(c->pw_nrm), st));
    }
    // the host-driven loop reports the residual relative to the whitened data
    ST_TRY(read_back(c, c->h_norms, c->pw_nrm.ptr, (size_t)P * sizeof(double), st));
    r.b0norm = sqrt(sum_host(c->h_norms, P));
    if (sigma0) HIP_TRY(launch_pwls_scale(r.sigma, P_<const float>(c->pw_dinv), Q, true, st));  // D sigma0
    r.lam_scale = P_<const float>(c->pw_dinv);
    r.op_gamma = P_<const float>(c->pw_g);
    r.op_eps = P_<const float>(c->pw_eps);
    r.op_B0 = P_<const float2>(c->pw_B0w);
  }
  return CLSIMG_OK;
}

// Table I on the device: one workgroup per outer step, the full-grid
// multiplier kernel between steps; the host only checks for the end.
int solve_device_loop(SolveRun& r) {
  clsimg_ctx* c = r.c;
  hipStream_t st = r.st;
  const clsimg_opts* o = r.o;
  OuterState* ost = P_<OuterState>(c->ostate);
  HIP_TRY(launch_outer_init(ost, r.dec, st));
  OuterParams op;
  op.st = ost;
  op.Flist = r.Flist;
  op.Ulist = r.Ulist;
  op.sigma = r.sigma;
  op.gamma = r.op_gamma;
  op.eps = r.op_eps;
  op.state = r.state;
  op.B0 = r.op_B0;
  op.Bb = r.Bb;
  op.E = r.E;
  op.keys = r.keys;
  op.nkeys = beam_grid(r.Q);
  op.tab = r.tab();
  op.P = r.P;
  op.Q = r.Q;
  op.atol = o->atol;
  op.btol = o->btol;
  op.conlim = o->conlim;
  op.itnlim = o->itnlim;
  op.max_outer = r.max_outer;
  op.max_f = hand_over_limit(o);
  op.Lw = r.pwls ? P_<const float2>(c->pw_Lw) : nullptr;
  op.rowscale = r.pwls ? P_<const float>(c->pw_rs) : nullptr;
  int nb = 8;
  for (;;) {
    for (int b = 0; b < nb; ++b) {
      HIP_TRY(launch_outer_step(op, st));
      HIP_TRY(launch_beam_lambda(nullptr, r.E, r.P, op.tab, &ost->lam_skip, r.state, r.keys, r.lam_scale, st));
    }
    ST_TRY(read_back(c, c->h_outer, ost, sizeof(OuterState), st));
    if (c->h_outer->done) break;
    nb = std::min(2 * nb, 128);
  }
  const OuterState& S = *c->h_outer;
  r.status = S.status == kStatusMaxOuter ? CLSIMG_WMAXOUTER : (S.status == kStatusCycle ? CLSIMG_WCYCLE : CLSIMG_OK);
  r.outer = S.outer;
  r.adds = S.adds;
  r.drops = S.drops;
  r.lsqr_total = S.lsqr_total;
  r.itnlim_hits = S.itnlim_hits;
  r.last_added = S.last_added;
  r.margin_lambda = S.margin_lambda;
  r.margin_z = S.margin_z;
  r.nF = S.nF;
  r.nU = S.nU;
  r.flops += S.psi_flops;
  // a free set too large for one workgroup: continue on the host from here
  r.host_loop = S.fallback != 0;
  r.dev_res2 = S.res2;
  r.dev_b0n2 = S.b0n2;
  return CLSIMG_OK;
}

// The full-grid multipliers of a feasible step (eqs. gls, etaL, etaU) from E
// and their argmin with the detection test; `fp32_only` takes the FP32
// kernels also in the reduced-precision modes.
int host_multipliers(SolveRun& r, bool fp32_only) {
  clsimg_ctx* c = r.c;
  hipStream_t st = r.st;
  const int P = r.P, Q = r.Q;
  if (r.pwls) fp32_only = true;  // PWLS: the multipliers in FP32, scaled by 1 / D_i
  if (r.beam_half && !fp32_only) {
    const bool bf = c->prec == CLSIMG_BF16;
    int* count = P_<int>(c->mx_count);
    HIP_TRY(launch_beam_lambda_refined(r.E, P, bf, r.tab(), r.grad_stop, r.state, c->frag_h.ptr,
                                       P_<float>(c->hscale), P_<double>(c->mx_abs), kCandAbsParts, r.keys,
                                       P_<float>(c->mx_lam), P_<int>(c->mx_cand), r.cand_cap, count, st,
                                       big_tiles(c, P), r.mult_stamps));
    // the candidates in FP32: Ut fragments of E from the correlation
    AdjParams ap = adj_params(c, r.g, P, r.frag_r, P_<const int>(c->mx_cand), r.cand_cap, r.grad_stop);
    ap.rows_part = P_<float>(c->part);
    ap.rows_cap = c->part.bytes / sizeof(float);
    ap.n_dev = count;
    HIP_TRY(launch_adjoint_lambda(ap, r.state, r.keys, st));
    HIP_TRY(launch_argmin_final(r.keys, (r.cand_cap + r.cand_tile - 1) / r.cand_tile, r.eps, r.state, r.dec, st,
                                count, r.cand_cap));
  } else if (r.beam_full_grid) {
    HIP_TRY(launch_beam_lambda(nullptr, r.E, P, r.tab(), r.grad_stop, r.state, r.keys, r.lam_scale, st));
    HIP_TRY(launch_argmin_final(r.keys, beam_grid(Q), r.op_eps, r.state, r.dec, st));
  } else if (r.beam_big_grid_ok) {
    HIP_TRY(launch_beam_prep_full(r.E, P, P_<float>(c->frag_b), st));
    HIP_TRY(launch_beam_big(3, P_<const float>(c->frag_b), r.tab(), r.grad_stop, nullptr, nullptr, 0.f, 0, 0, 1.f,
                            r.state, r.keys, st, fp32_only ? Stamps{} : r.mult_stamps, big_tiles(c, P),
                            r.lam_scale));
    HIP_TRY(launch_argmin_final(r.keys, beam_big_grid(P, Q, big_tiles(c, P)), r.op_eps, r.state, r.dec, st));
  } else {
    if (r.pwls) return CLSIMG_ENOTSUP;
    HIP_TRY(launch_adjoint_lambda(adj_params(c, r.g, P, r.frag_r, nullptr, Q, r.grad_stop), r.state, r.keys, st));
    HIP_TRY(launch_argmin_final(r.keys, r.ntiles_Q, r.eps, r.state, r.dec, st));
  }
  return CLSIMG_OK;
}

// One subproblem of the host-driven loop (eqs. subproblemLS, bsubproblemLS)
// by LSQR, the step of Table I and, after a feasible step, the multipliers.
int host_subproblem(SolveRun& r) {
  clsimg_ctx* c = r.c;
  const clsimg_opts* o = r.o;
  hipStream_t st = r.st;
  const int P = r.P, Q = r.Q, MT = r.MT;
  const bool fused = r.fused;
  if (r.outer >= r.max_outer) {
    r.status = CLSIMG_WMAXOUTER;
    r.stop = true;
    return CLSIMG_OK;
  }
  ST_TRY(compact(c, r.state, Q, st));
  // b = B0 - Psi_U gamma_U  (eq. bsubproblemLS); b = B0 while U is empty
  const float2* bsub = r.B0;
  if (r.nU > 0) {
    ST_TRY(correlate(c, r.g, P, r.Ulist, r.gamma, 1, r.nU, r.Bb, r.B0, -1.f, 1.f, nullptr, nullptr, nullptr, nullptr,
                     st));
    bsub = r.Bb;
  }
  r.flops += corr_flops(P, r.nU);
  // PWLS (eq. preWLS): the subproblem in whitened variables, L^-1 b L^-H with
  // the bound D gamma for D sigma (sum_U gamma_i a_i a_i^H whitens to the
  // same terms with D gamma and the whitened rows)
  const double2* Li = P_<const double2>(c->Li);
  if (r.pwls) {
    if (!fused) return CLSIMG_ENOTSUP;
    if (r.nU > 0) {
      HIP_TRY(launch_pwls_sandwich(Li, bsub, P, false, P_<double2>(c->pw_T), P_<float2>(c->pw_Bw), nullptr, st));
      bsub = P_<const float2>(c->pw_Bw);
    } else {
      bsub = r.op_B0;
    }
  }
  const int nF = r.nF;
  if (fused) {
    // the cache grows geometrically with |F| (a reallocation synchronises the device)
    size_t cap = 256;
    while (cap < (size_t)nF) cap *= 2;
    ST_TRY(ensure(c, c->xf, cap * 2 * pad_p(P) * sizeof(float)));
    r.xf = P_<float>(c->xf);
    HIP_TRY(launch_xf(r.tab(), r.Flist, nF, r.xf, st));
    if (r.pwls) HIP_TRY(launch_pwls_xf_whiten(Li, P, r.Flist, nF, P_<const float>(c->pw_rs), r.xf, st));
  }
  const int nalpha = ntiles_adj(P, nF);
  const int nalpha2 = (nF + adjoint_lsqr2_tile_width(MT, nF) - 1) / adjoint_lsqr2_tile_width(MT, nF);
  int it = 1;
  // LSQR engine: one workgroup when the subproblem fits in its LDS (no grid
  // barriers at all), else one cooperative kernel, else two kernels per
  // step (P <= 96), else the split-K correlation with separate reductions
  const int want = o->lsqr_engine;
  const bool one_cu = fused && (want == CLSIMG_LSQR_AUTO || want == CLSIMG_LSQR_ONE_WG) && lsqr_cu_fits(P, nF);
  // (above 48 antennas the two-kernel step is the faster one: 7.7 against
  // 10.7 ms for a 56-antenna solve, 17.3 against 24.7 ms at 64 antennas)
  const bool coop_auto = want == CLSIMG_LSQR_AUTO && MT <= 6;
  const bool persist = !one_cu && fused && c->coop && (coop_auto || want == CLSIMG_LSQR_COOP) &&
                       persist_fits(P, nF);
  if (nF > 0) {
    const int itnlim = o->itnlim < 0 ? 4 * nF + 100 : o->itnlim;
    if (one_cu) {
      HIP_TRY(launch_lsqr_setup2(r.S2, r.done, r.bar, r.lerr, o->atol, o->btol, o->conlim, itnlim, st));
      LsqrCuParams lc;
      lc.P = P;
      lc.n = nF;
      lc.xf = r.xf;
      lc.B = bsub;
      lc.x_out = r.x;
      lc.Sfinal = r.Sfin;
      lc.done = r.done;
      lc.atol = o->atol;
      lc.btol = o->btol;
      lc.conlim = o->conlim;
      lc.itnlim = itnlim;
      HIP_TRY(launch_lsqr_cu(lc, st));
    } else if (persist) {
      // the whole LSQR solve in one cooperative kernel
      HIP_TRY(launch_lsqr_setup2(r.S2, r.done, r.bar, r.lerr, o->atol, o->btol, o->conlim, itnlim, st));
      LsqrPersistParams lp;
      lp.MT = MT;
      lp.P = P;
      lp.n = nF;
      lp.ntp = MT * (MT + 1) / 2;
      lp.xf = r.xf;
      lp.B = bsub;
      lp.frag = r.frag_u;
      lp.pbeta = r.bparts[0];
      lp.palpha = r.alpha_part;
      lp.vraw = r.vraw;
      lp.x_out = r.x;
      lp.Sfinal = r.Sfin;
      lp.done = r.done;
      lp.bar = r.bar;
      lp.err = r.lerr;
      lp.atol = o->atol;
      lp.btol = o->btol;
      lp.conlim = o->conlim;
      lp.itnlim = itnlim;
      HIP_TRY(launch_lsqr_persist(lp, st));
    } else if (fused) {
      // beta_1 u_1 = b ; alpha_1 v_1 = Psi_F^H u_1  (eqs. initbeta, initu); then step 1
      HIP_TRY(launch_lsqr_setup(r.S2, r.done, o->atol, o->btol, o->conlim, itnlim, st));
      ST_TRY(correlate(c, r.g, P, nullptr, nullptr, 0, 0, r.u, bsub, 0.f, 1.f, nullptr, r.frag_u, r.bparts[1],
                       nullptr, st));
      HIP_TRY(launch_adjoint_lsqr2(r.lsqr_adj(r.done), EpiLsqrV2{r.vraw, r.v, r.bparts[1], r.nbeta, r.alpha_part, 1},
                                   st));
      HIP_TRY(launch_lsqr_fwd(r.fwd_params(1, nalpha2), st));
    } else {
      ST_TRY(correlate(c, r.g, P, nullptr, nullptr, 0, 0, r.u, bsub, 0.f, 1.f, nullptr, r.frag_u, r.beta_part,
                       nullptr, st));
      HIP_TRY(launch_adjoint_lsqr(r.lsqr_adj_rows(nullptr), r.v, r.beta_part, r.nbeta, r.alpha_part, 1, st));
      HIP_TRY(launch_lsqr_init_scalars(r.ls, r.beta_part, r.nbeta, r.alpha_part, nalpha, r.v, r.w, r.x, nF, o->atol,
                                       o->btol, o->conlim, itnlim, st));
    }
  }
  for (;;) {
    if (nF > 0 && !persist && !one_cu) {
      for (int b = 0; b < r.batch; ++b) {
        // beta u <- Psi_F v - alpha u ; alpha v <- Psi_F^H u - beta v  (eq. lanczos)
        if (fused) {
          HIP_TRY(launch_adjoint_lsqr2(r.lsqr_adj(r.done),
                                       EpiLsqrV2{r.vraw, r.v, r.bparts[(it + 1) & 1], r.nfw, r.alpha_part, 0}, st));
          ++it;
          HIP_TRY(launch_lsqr_fwd(r.fwd_params(it, nalpha2), st));
        } else {
          ST_TRY(correlate(c, r.g, P, r.Flist, r.v, 0, nF, r.u, r.u, 1.f, 0.f, r.ls, r.frag_u, r.beta_part,
                           r.lsqr_stop, st));
          const AdjParams ap = r.lsqr_adj_rows(r.lsqr_stop);
          if (adjoint_lsqr_fuses(ap)) {  // the whole list in one epilogue workgroup: the step there too
            HIP_TRY(launch_adjoint_lsqr_step(ap, r.v, r.beta_part, r.nbeta, r.alpha_part, r.ls, r.w, r.x, st));
          } else {
            HIP_TRY(launch_adjoint_lsqr(ap, r.v, r.beta_part, r.nbeta, r.alpha_part, 0, st));
            HIP_TRY(launch_lsqr_update(r.ls, r.beta_part, r.nbeta, r.alpha_part, nalpha, r.v, r.w, r.x, nF, st));
          }
        }
      }
    }
    if (persist || one_cu)
      HIP_TRY(launch_step(r.done, r.lerr, r.Sfin, r.x, r.x, r.Flist, nF, r.sigma, r.op_gamma, r.state, r.dec, st));
    else if (fused)
      HIP_TRY(launch_step(r.done, nullptr, r.Sfin, r.x, r.x1, r.Flist, nF, r.sigma, r.op_gamma, r.state, r.dec, st));
    else
      HIP_TRY(launch_step(r.lsqr_stop, nullptr, r.ls, r.x, r.x, r.Flist, nF, r.sigma, r.op_gamma, r.state, r.dec,
                          st));
    // gradient on the active pixels, only after a feasible subproblem (eq. gls):
    // E = Psi_F sigma_F - b, then g = Psi^H E on every pixel
    if (fused) {
      CorrOsParams cp;
      cp.MT = MT;
      cp.P = P;
      cp.xf = r.xf;
      cp.n = nF;
      cp.vals = r.sigma;
      cp.gidx = r.Flist;
      cp.out = r.pwls ? P_<float2>(c->pw_Eh) : r.E;
      cp.B = bsub;
      cp.cK = 1.f;
      cp.cB = -1.f;
      cp.frag = r.frag_r;
      cp.stop_flag = r.grad_stop;
      HIP_TRY(launch_corr_os(cp, st));
      // PWLS: the multiplier of pixel i is a_i^H (L^-H E L^-1) a_i / D_i
      if (r.pwls)
        HIP_TRY(launch_pwls_sandwich(Li, P_<const float2>(c->pw_Eh), P, true, P_<double2>(c->pw_T), r.E, nullptr, st));
    } else {
      ST_TRY(correlate(c, r.g, P, r.Flist, r.sigma, 1, nF, r.E, bsub, 1.f, -1.f, nullptr, r.frag_r, nullptr,
                       r.grad_stop, st));
    }
    ST_TRY(host_multipliers(r, false));
    ST_TRY(read_back(c, c->h_dec, r.dec, sizeof(SolveDecision), st));
    const bool grad = c->h_dec->lsqr_done && c->h_dec->feasible;
    if (r.mult_stamps.start && grad && (r.beam_half || !r.beam_full_grid)) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, c->tm_ev[0], c->tm_ev[1]));
      c->tm_ms += ms;
      ++c->tm_n;
    }
    if (r.beam_half && grad && c->h_dec->cand_overflow) {
      // more candidates than the list holds: this step's multipliers in FP32
      ST_TRY(host_multipliers(r, true));
      ST_TRY(read_back(c, c->h_dec, r.dec, sizeof(SolveDecision), st));
      if (o->trace) fprintf(stderr, "clsimg: outer %d: candidate list full, multipliers in FP32\n", r.outer);
    }
    if (c->h_dec->lsqr_done) break;
    if (persist || one_cu || c->h_dec->lsqr_err) return CLSIMG_EHIP;  // LSQR kernel did not finish
    r.batch = std::min(r.batch * 2, 64);
  }
  const SolveDecision d = *c->h_dec;
  if (o->trace) {
    ST_TRY(read_back(c, c->h_lsqr, fused ? r.Sfin : r.ls, sizeof(LsqrState), st));
    const LsqrState& L = *c->h_lsqr;
    fprintf(stderr,
            "clsimg: outer %d nF %d nU %d itn %d istop %d alpha %.3e beta %.3e rnorm %.3e "
            "arnorm %.3e anorm %.3e acond %.3e xnorm %.3e bnorm %.3e feasible %d ib %d mu %.3e "
            "i_min %d lam %.4e eps %.4e\n",
            r.outer, nF, r.nU, L.itn, L.istop, L.alpha, L.beta, L.rnorm, L.arnorm, L.anorm, L.acond, L.xnorm, L.bnorm,
            d.feasible, d.ib, (double)d.mu_max, d.i_min, (double)d.lam_min, (double)d.eps_min);
  }
  r.batch = std::max(2, std::min(64, d.lsqr_itn + 1));
  ++r.outer;
  r.lsqr_total += d.lsqr_itn;
  if (nF > 0) r.flops += beam_flops(P, nF) + d.lsqr_itn * (corr_flops(P, nF) + beam_flops(P, nF));
  if (d.feasible) r.flops += corr_flops(P, nF) + beam_flops(P, Q);
  if (nF > 0 && d.lsqr_istop == 7) ++r.itnlim_hits;
  if (d.feasible) {
    r.need_solve = false;
    if (nF > 0) r.margin_z = std::min(r.margin_z, (double)d.margin_z);
    if (d.i_min < 0) {  // no active pixel left
      r.stop = true;
      return CLSIMG_OK;
    }
    r.lam_min = d.lam_min;
    r.eps_min = d.eps_min;
    r.i_min = d.i_min;
    r.st_min = d.st_min;
  } else {
    ++r.drops;
    --r.nF;
    if (d.ib_to == CLSIMG_STATE_U) ++r.nU;
    r.need_solve = true;
    if (d.ib == r.last_added && d.mu_max == 0.0f) {
      r.status = CLSIMG_WCYCLE;
      r.stop = true;
      return CLSIMG_OK;
    }
  }
  r.last_added = -1;
  return CLSIMG_OK;
}

// Table I driven from the host: subproblems, and after each feasible one the
// detection test on the most negative multiplier (release into F or stop).
int solve_host_loop(SolveRun& r) {
  while (!r.stop) {
    if (r.need_solve) {
      ST_TRY(host_subproblem(r));
      continue;
    }
    if (r.eps_min > 0.f) r.margin_lambda = std::min(r.margin_lambda, fabs((double)r.lam_min + r.eps_min) / r.eps_min);
    if (!(r.lam_min < -r.eps_min)) break;
    HIP_TRY(launch_set_state(r.state, r.i_min, (uint8_t)CLSIMG_STATE_F, r.st));
    ++r.adds;
    ++r.nF;
    if (r.st_min == CLSIMG_STATE_U) --r.nU;
    r.last_added = r.i_min;
    r.need_solve = true;
  }
  return CLSIMG_OK;
}

// The two-kernel LSQR over the free-set cache r.xf (P <= 96) run to the end
// on its own: steps enqueued in growing batches with the done flag read back
// between them; the solution left in r.x.
int lsqr_fused_solve(SolveRun& r, const float2* bsub, int itnlim) {
  clsimg_ctx* c = r.c;
  const clsimg_opts* o = r.o;
  hipStream_t st = r.st;
  const int nF = r.nF, tw = adjoint_lsqr2_tile_width(r.MT, nF);
  const int nalpha2 = (nF + tw - 1) / tw;
  HIP_TRY(launch_lsqr_setup(r.S2, r.done, o->atol, o->btol, o->conlim, itnlim, st));
  ST_TRY(correlate(c, r.g, r.P, nullptr, nullptr, 0, 0, r.u, bsub, 0.f, 1.f, nullptr, r.frag_u, r.bparts[1], nullptr,
                   st));
  HIP_TRY(launch_adjoint_lsqr2(r.lsqr_adj(r.done), EpiLsqrV2{r.vraw, r.v, r.bparts[1], r.nbeta, r.alpha_part, 1}, st));
  int it = 1, batch = 4;
  HIP_TRY(launch_lsqr_fwd(r.fwd_params(1, nalpha2), st));
  for (;;) {
    ST_TRY(read_back(c, c->h_status, r.done, sizeof(int), st));
    if (*c->h_status) break;
    if (it > itnlim + 256) return CLSIMG_EHIP;  // LSQR stops itself at itnlim
    for (int b = 0; b < batch; ++b) {
      HIP_TRY(launch_adjoint_lsqr2(r.lsqr_adj(r.done),
                                   EpiLsqrV2{r.vraw, r.v, r.bparts[(it + 1) & 1], r.nfw, r.alpha_part, 0}, st));
      ++it;
      HIP_TRY(launch_lsqr_fwd(r.fwd_params(it, nalpha2), st));
    }
    batch = std::min(batch * 2, 64);
  }
  HIP_TRY(launch_lsqr_pick(r.Sfin, r.x1, r.x, nF, st));
  return CLSIMG_OK;
}

// Statistics; after the host-driven loop the final residual ||B0 - Psi sigma||_F
// is formed from the final sets (the device loop keeps that of its last
// feasible step, which is the final image).
int solve_stats(SolveRun& r, clsimg_stats* stats) {
  clsimg_ctx* c = r.c;
  if (r.status == CLSIMG_OK && r.itnlim_hits) r.status = CLSIMG_WITNLIM;
  double res2 = r.dev_res2;
  const double b0n2 = r.dev_b0n2;
  if (r.host_loop) {
    ST_TRY(compact(c, r.state, r.Q, r.st));
    ST_TRY(read_back(c, c->h_dec, r.dec, sizeof(SolveDecision), r.st));
    r.nF = c->h_dec->nF;
    r.nU = c->h_dec->nU;
    ST_TRY(correlate(c, r.g, r.P, r.Ulist, r.gamma, 1, r.nU, r.Bb, r.B0, -1.f, 1.f, nullptr, nullptr, nullptr,
                     nullptr, r.st));
    ST_TRY(correlate(c, r.g, r.P, r.Flist, r.sigma, 1, r.nF, r.E, r.Bb, 1.f, -1.f, nullptr, nullptr, r.beta_part,
                     nullptr, r.st));
    if (r.pwls) {  // PWLS: the residual of the whitened problem, L^-1 (Psi sigma - b) L^-H
      HIP_TRY(launch_pwls_sandwich(P_<const double2>(c->Li), r.E, r.P, false, P_<double2>(c->pw_T),
                                   P_<float2>(c->pw_Eh), P_<double>(c->pw_nrm), r.st));
      ST_TRY(read_back(c, c->h_norms, c->pw_nrm.ptr, (size_t)r.P * sizeof(double), r.st));
      res2 = sum_host(c->h_norms, r.P);
    } else {
      ST_TRY(read_back(c, c->h_norms, r.beta_part, r.nbeta * sizeof(double), r.st));
      res2 = sum_host(c->h_norms, r.nbeta);
    }
    r.flops += corr_flops(r.P, r.nU) + corr_flops(r.P, r.nF);
  }
  stats->status = r.status;
  stats->outer_iters = r.outer;
  stats->adds = r.adds;
  stats->drops = r.drops;
  stats->lsqr_iters_total = r.lsqr_total;
  stats->lsqr_itnlim_hits = r.itnlim_hits;
  stats->nF = r.nF;
  stats->nU = r.nU;
  if (r.host_loop) {
    const double rn = sqrt(res2);
    stats->rel_residual = r.b0norm > 0 ? rn / r.b0norm : 0.0;
    stats->objective = 0.5 * rn * rn;
  } else {
    stats->rel_residual = b0n2 > 0.0 ? sqrt(res2 / b0n2) : 0.0;
    stats->objective = 0.5 * res2;
  }
  stats->min_margin_lambda = r.margin_lambda;
  stats->min_margin_z = r.margin_z;
  stats->psi_flops = r.flops;
  return r.status;
}

}  // namespace

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
  SolveRun r;
  r.c = c;
  r.g = g;
  r.o = o;
  r.st = (hipStream_t)stream;
  r.P = a->P;
  r.Q = g->nl * g->nm;
  r.sigma = sigma;
  r.state = state;
  ST_TRY(solve_setup(r, R, a, noise_diag, sigma0, state0, mf_out, gamma_out));
  if (r.device_loop) ST_TRY(solve_device_loop(r));
  if (r.host_loop) ST_TRY(solve_host_loop(r));
  // PWLS solves for D sigma: sigma = D^-1 (D sigma)
  if (r.pwls) HIP_TRY(launch_pwls_scale(r.sigma, P_<const float>(c->pw_dinv), r.Q, false, r.st));
  return solve_stats(r, stats);
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
    ST_TRY(ensure(c, c->hscale, kHalfScaleFloats * sizeof(float)));
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
  ST_TRY(compact(c, state, Q, st));
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
      ST_TRY(compact(c, state, Q, st));
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
  ST_TRY(compact(c, state, Q, st));
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
  // the shifted steering rows live in the free-set cache of the LSQR engines
  // that read it (up to 12 row tiles, P <= 96)
  if (o->cost != CLSIMG_COST_LS || MT > 12 || !beam_any(P)) return CLSIMG_ENOTSUP;
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
  // the cooperative and the two-kernel LSQR (free sets beyond one workgroup)
  const int nparts = std::max(std::max(reduce_blocks(P), lsqr_fwd_waves(P)), Q / 32 + 64);
  ST_TRY(ensure(c, c->bpart0, (size_t)nparts * sizeof(double)));
  ST_TRY(ensure(c, c->bpart1, (size_t)nparts * sizeof(double)));
  ST_TRY(ensure(c, c->alpha_part, (size_t)(Q / 16 + 64) * sizeof(double)));
  for (DevBuf* b : {&c->v, &c->w, &c->x1, &c->w1, &c->vraw}) ST_TRY(ensure(c, *b, (size_t)Q * sizeof(float)));
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

  // the two-kernel LSQR's operands (its steering rows: the shifted cache)
  SolveRun fr;
  fr.c = c;
  fr.g = g;
  fr.o = o;
  fr.st = st;
  fr.P = P;
  fr.Q = Q;
  fr.MT = MT;
  fr.nbeta = reduce_blocks(P);
  fr.nfw = lsqr_fwd_waves(P);
  fr.Flist = Flist;
  fr.xf = xf;
  fr.u = P_<float2>(c->u);
  fr.v = P_<float>(c->v);
  fr.w = P_<float>(c->w);
  fr.x = x;
  fr.x1 = P_<float>(c->x1);
  fr.w1 = P_<float>(c->w1);
  fr.vraw = P_<float>(c->vraw);
  fr.frag_u = P_<float>(c->frag_u);
  fr.alpha_part = P_<double>(c->alpha_part);
  fr.bparts[0] = P_<double>(c->bpart0);
  fr.bparts[1] = P_<double>(c->bpart1);
  fr.S2 = S2;
  fr.Sfin = Sfin;
  fr.done = done;
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
      ST_TRY(compact(c, state, Q, st));
      HIP_TRY(launch_offgrid_sets(state, Q, gamma0, offsets, sigma, st));
      ST_TRY(read_back(c, c->h_dec, dec, sizeof(SolveDecision), st));
      nF = c->h_dec->nF;
      nU = c->h_dec->nU;
      // LSQR in one workgroup when the subproblem fits its LDS, else in one
      // cooperative kernel (up to 48 antennas), else two kernels per step
      const bool one_cu = lsqr_cu_fits(P, nF);
      const bool persist = !one_cu && c->coop && pad_p(P) / 8 <= 6 && persist_fits(P, nF);
      fr.nF = nF;
      // b = B0 - Psi_U gamma0_U on the grid (eq. bsubproblemLS)
      ST_TRY(correlate(c, g, P, Ulist, gamma0, 1, nU, Bb, B0, -1.f, 1.f, nullptr, nullptr, nullptr, nullptr, st));
      flops += corr_flops(P, nU);
      const int itnlim = o->itnlim < 0 ? 4 * nF + 100 : o->itnlim;
      for (int t = 0; t <= rounds; ++t) {
        HIP_TRY(xf_off(nF));
        HIP_TRY(launch_lsqr_setup2(S2, done, bar, lerr, o->atol, o->btol, o->conlim, itnlim, st));
        if (nF > 0 && one_cu) {
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
        } else if (nF > 0 && persist) {
          LsqrPersistParams lp;
          lp.MT = MT;
          lp.P = P;
          lp.n = nF;
          lp.ntp = MT * (MT + 1) / 2;
          lp.xf = xf;
          lp.B = Bb;
          lp.frag = P_<float>(c->frag_u);
          lp.pbeta = P_<double>(c->bpart0);
          lp.palpha = P_<double>(c->alpha_part);
          lp.vraw = P_<float>(c->vraw);
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
        } else if (nF > 0) {
          ST_TRY(lsqr_fused_solve(fr, Bb, itnlim));
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
      if (beam_fits(P)) {
        HIP_TRY(launch_beam_lambda(nullptr, E, P, tab, grad_stop, state, keys, nullptr, st));
        HIP_TRY(launch_argmin_final(keys, beam_grid(Q), eps, state, dec, st));
      } else {
        HIP_TRY(launch_beam_prep_full(E, P, P_<float>(c->frag_b), st));
        HIP_TRY(launch_beam_big(3, P_<const float>(c->frag_b), tab, grad_stop, nullptr, nullptr, 0.f, 0, 0, 1.f, state,
                                keys, st, Stamps{}, big_tiles(c, P)));
        HIP_TRY(launch_argmin_final(keys, beam_big_grid(P, Q, big_tiles(c, P)), eps, state, dec, st));
      }
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
  ST_TRY(compact(c, state, Q, st));
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

}  // extern "C"

namespace {

// Step pairs in one captured round of a batched solve: the loop replays the
// round 1, 2, 4 ... 16 times between its looks at the requests' states.
constexpr int kRoundPairs = 8;

// The captured round (kRoundPairs outer-step and multiplier launches for all
// requests), built once per (parameter arrays, batch size, P) on a private
// stream; its kernels read every per-step value from device memory, so one
// graph serves every round and every call with the same arguments.
int batch_round_graph(clsimg_ctx* c, const OuterParams* dp, const BeamLamItem* di, int n, int bpr, int P) {
  if (c->round_exec && c->round_key[0] == dp && c->round_key[1] == di && c->round_key_n == n &&
      c->round_key_bpr == bpr && c->round_key_P == P)
    return CLSIMG_OK;
  if (c->round_exec) {
    HIP_TRY(hipGraphExecDestroy(c->round_exec));
    c->round_exec = nullptr;
  }
  if (!c->cap_st) HIP_TRY(hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int b = 0; b < kRoundPairs && e == hipSuccess; ++b) {
    e = launch_outer_step_batch(dp, n, P, c->cap_st);
    if (e == hipSuccess) e = launch_beam_lambda_batch(di, n, bpr, P, c->cap_st);
  }
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(c->cap_st, &graph);
  if (e == hipSuccess) e = ee;
  if (e == hipSuccess) e = hipGraphInstantiate(&c->round_exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  HIP_TRY(e);
  c->round_key[0] = dp;
  c->round_key[1] = di;
  c->round_key_n = n;
  c->round_key_bpr = bpr;
  c->round_key_P = P;
  return CLSIMG_OK;
}

}  // namespace

extern "C" {

namespace {
// one request solved alone, as clsimg_solve does it; the worse of two codes
int solve_request_alone(clsimg_ctx* c, clsimg_request& q, const clsimg_opts* o, void* stream) {
  return clsimg_solve(c, q.R, &q.array, &q.grid, q.noise_diag, o, nullptr, nullptr, q.sigma, q.state, q.mf, q.gamma,
                      &q.stats, stream);
}
int worse_status(int worst, int status) {
  if (status < 0) return worst < 0 ? worst : status;
  return (worst >= 0 && status > worst) ? status : worst;
}
int solve_batch_device(clsimg_ctx* c, int32_t n, clsimg_request* reqs, const clsimg_opts* o, void* stream);
}  // namespace

int clsimg_solve_batch(clsimg_ctx* c, int32_t n, clsimg_request* reqs, const clsimg_opts* o, void* stream) {
  if (!c || !reqs || n < 1) return CLSIMG_EINVAL;
  for (int r = 0; r < n; ++r) memset(&reqs[r].stats, 0, sizeof(clsimg_stats));
  for (int r = 0; r < n; ++r) {
    if (!reqs[r].R || !reqs[r].sigma || !reqs[r].state) return CLSIMG_EINVAL;
    ST_TRY(check_opts(o, reqs[r].array.P));
    ST_TRY(check_geometry(&reqs[r].array, &reqs[r].grid));
  }
  const int P = reqs[0].array.P;
  bool one_p = true;
  for (int r = 1; r < n; ++r) one_p = one_p && reqs[r].array.P == P;
  if (!one_p) {
    // several array sizes: one batch per size, in order of first appearance
    std::vector<int> sizes;
    for (int r = 0; r < n; ++r)
      if (std::find(sizes.begin(), sizes.end(), reqs[r].array.P) == sizes.end()) sizes.push_back(reqs[r].array.P);
    int worst = CLSIMG_OK;
    std::vector<clsimg_request> group;
    for (int sz : sizes) {
      group.clear();
      for (int r = 0; r < n; ++r)
        if (reqs[r].array.P == sz) group.push_back(reqs[r]);
      const int st = clsimg_solve_batch(c, (int32_t)group.size(), group.data(), o, stream);
      for (int r = 0, k = 0; r < n; ++r)
        if (reqs[r].array.P == sz) reqs[r].stats = group[k++].stats;
      if (st < 0 && st != CLSIMG_ENOTSUP && st != CLSIMG_ENOTPD) return st;  // a call-level failure
      worst = worse_status(worst, st);
    }
    return worst;
  }
  if (!request_on_device(P)) {
    // beyond the device-resident loop: the requests one after another on the
    // host-driven loop, each exactly its solve alone
    int worst = CLSIMG_OK;
    for (int r = 0; r < n; ++r) worst = worse_status(worst, solve_request_alone(c, reqs[r], o, stream));
    return worst;
  }
  const int st = solve_batch_device(c, n, reqs, o, stream);
  int handed = 0;
  for (int r = 0; r < n; ++r) handed += reqs[r].stats.status == CLSIMG_ENOTSUP;
  if (st < 0 && !(st == CLSIMG_ENOTSUP && handed)) return st;
  // a request whose free set outgrew the device loop (or passed hand_over_free)
  // is solved again alone: the device loop hands it over to the host loop at
  // the same step
  int worst = CLSIMG_OK;
  for (int r = 0; r < n; ++r) {
    const int status = reqs[r].stats.status == CLSIMG_ENOTSUP ? solve_request_alone(c, reqs[r], o, stream)
                                                               : reqs[r].stats.status;
    worst = worse_status(worst, status);
  }
  return worst;
}

namespace {
int solve_batch_device(clsimg_ctx* c, int32_t n, clsimg_request* reqs, const clsimg_opts* o, void* stream) {
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
                     o->precision == CLSIMG_FP32;
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

  if (o->batch_graph) ST_TRY(batch_round_graph(c, dp, di, n, bpr, P));
  int nb = 8;
  for (;;) {
    if (o->batch_graph) {
      for (int b = 0; b < nb; b += kRoundPairs) HIP_TRY(hipGraphLaunch(c->round_exec, st));
    } else {
      for (int b = 0; b < nb; ++b) {
        HIP_TRY(launch_outer_step_batch(dp, n, P, st));
        HIP_TRY(launch_beam_lambda_batch(di, n, bpr, P, st));
      }
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
  for (int r = 0; r < n; ++r) worst = worse_status(worst, request_finish(reqs[r], o, slice(r), L, hs[r], st));
  return worst;
}
}  // namespace

}  // extern "C"
