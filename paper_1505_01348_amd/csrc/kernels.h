// Parameter blocks, epilogues and host launchers of the clsimg kernels.
#pragma once

#include "common.h"

namespace clsimg {

// Device-resident LSQR scalars (FP64), Sec. IV-A with the LSQR updates.
struct LsqrState {
  double alpha, beta;        // current alpha_i, beta_i
  double rhobar, phibar;     // rotation state
  double bnorm, anorm2, ddnorm;
  double rnorm, arnorm, anorm, acond, xnorm;
  double atol, btol, conlim;
  int itn, itnlim, istop, done;
};

struct AdjParams {
  const float* frag;  // Ut fragments, 4 Pp^2 floats (used when U is NULL)
  const float2* U;    // or: complex P x P matrix, staged into fragments by the kernel
  const float* xf;    // optional: real-embedded steering vectors of the listed pixels,
                      // 2Pp floats per list position (else generated from the tables)
  int P, MT, KS;
  Tables tab;
  const int* idx;     // output column k looks at pixel idx[k] (NULL: pixel k)
  int n;
  const int* stop_flag;
  // K covariance blocks summed in one launch: block k uses frag + k * frag_stride
  // and the tables at El/Em + k * tab_stride (fragment input only)
  int nblk = 1;
  size_t frag_stride = 0, tab_stride = 0;
  // 1: one block per workgroup (blockIdx.y = block), for epilogues that keep
  // the blocks apart; 0: every workgroup adds the column dots of all blocks
  int blk_grid = 0;
  // optional workspace (rows_cap floats) for the row-split beamformer of large
  // arrays (LSQR adjoint beyond 12 row tiles, fragment input): one partial
  // column dot per group of four row tiles and listed pixel
  float* rows_part = nullptr;
  size_t rows_cap = 0;
  // optional: the list length on the device (at most n), for lists built by a
  // kernel; columns from *n_dev on are left out (row-split beamformer only)
  const int* n_dev = nullptr;
};

struct FwdParams {
  Tables tab;
  int MT;
  const int* idx;     // k-th term uses pixel idx[k] (NULL: pixel k)
  const float* vals;  // weight of the k-th term: gather ? vals[pixel] : vals[k]
  int gather;
  int n;
  int chw;            // pixels per workgroup, a multiple of 16
  float* part;
  const int* stop_flag;
  // K covariance blocks in one launch (blockIdx.z): block k reads the tables
  // at El/Em + k * tab_stride and writes its partials at part + k * part_stride
  int nblk = 1;
  size_t tab_stride = 0, part_stride = 0;
};

struct RedParams {
  const float* part;
  int nchunks, MT, P;
  float2* out;
  const float2* B;
  float cK, cB;
  const LsqrState* lsqr;  // if set: cB = -alpha/beta
  float* frag;            // optional Ut fragments of out
  double* norm_part;      // optional per-block sum |out|^2
  const int* stop_flag;
  // K covariance blocks in one launch (blockIdx.y): block k adds k * stride to
  // part, out, B, frag and norm_part
  int nblk = 1;
  size_t part_stride = 0, out_stride = 0, B_stride = 0, frag_stride = 0, norm_stride = 0;
};

struct LsqrFwdParams {
  Tables tab;
  int MT, P;
  const int* Flist;
  int n;
  LsqrState* S;            // two slots, by iteration parity
  LsqrState* Sfinal;       // the state of the last step, written when it stops
  int* done;               // set once the stopping tests pass
  int it;                  // this launch finishes step it-1 and starts step it
  const float* vraw;       // unnormalised v from the beamforming of step it-1
  float* vnorm;            // v_it (written by workgroup 0)
  const double* alpha_part;
  int nalpha;
  const double* beta_in;   // ||u_it||^2 partials
  int nbeta_in;
  double* beta_out;        // ||u_{it+1}||^2 partials, one per wave
  float *x0, *x1, *w0, *w1;
  const float* xf;         // steering vectors of the free set
  float2* u;               // unnormalised u, updated in place
  float* frag;             // Ut fragments of the new u
  int ntp;                 // upper-triangle tiles MT(MT+1)/2
};

// ---- adjoint epilogues: called by every thread of the block once per tile --
struct NoCtx {};

struct EpiStore {
  float* out;
  float scale;
  using Ctx = NoCtx;
  using Pre = NoCtx;
  __device__ Ctx init() const { return {}; }
  __device__ Pre prefetch(int, bool) const { return {}; }
  __device__ void operator()(int, int col, int, float g, bool ok, const Ctx&, const Pre&) const {
    if (ok) out[col] = g * scale;
  }
};

// column dots of covariance block blockIdx.y at out + blockIdx.y * stride
struct EpiStoreBlk {
  float* out;
  size_t stride;
  using Ctx = NoCtx;
  using Pre = NoCtx;
  __device__ Ctx init() const { return {}; }
  __device__ Pre prefetch(int, bool) const { return {}; }
  __device__ void operator()(int, int col, int, float g, bool ok, const Ctx&, const Pre&) const {
    if (ok) out[blockIdx.y * stride + col] = g;
  }
};

struct EpiMF {
  float* mf;
  float* eps;
  float eps_scale;
  using Ctx = NoCtx;
  using Pre = NoCtx;
  __device__ Ctx init() const { return {}; }
  __device__ Pre prefetch(int, bool) const { return {}; }
  __device__ void operator()(int, int col, int, float g, bool ok, const Ctx&, const Pre&) const {
    if (ok) {
      mf[col] = g;
      if (eps) eps[col] = g * eps_scale;
    }
  }
};

struct EpiMVDR {
  float* gamma;
  double C, kb_coef;
  using Ctx = NoCtx;
  using Pre = NoCtx;
  __device__ Ctx init() const { return {}; }
  __device__ Pre prefetch(int, bool) const { return {}; }
  __device__ void operator()(int, int col, int, float g, bool ok, const Ctx&, const Pre&) const {
    if (ok) {
      const double h = (double)g;
      gamma[col] = (float)(C / h + kb_coef / h);
    }
  }
};

// Lagrange multipliers of the active pixels (eqs. etaL / etaU) and a per-tile
// argmin key (ordered value << 32 | pixel): ties go to the lowest pixel.
struct EpiLambda {
  const uint8_t* state;
  uint64_t* part;
  using Ctx = NoCtx;
  using Pre = NoCtx;
  __device__ Ctx init() const { return {}; }
  __device__ Pre prefetch(int, bool) const { return {}; }
  __device__ void operator()(int tile, int, int pix, float g, bool ok, const Ctx&, const Pre&) const {
    __shared__ uint64_t sh[8];
    uint64_t key = ~0ull;
    if (ok) {
      const uint8_t s = state[pix];
      if (s != 1) {
        const float lam = (s == 0) ? g : -g;
        key = ((uint64_t)ordered_bits(lam) << 32) | (uint32_t)pix;
      }
    }
    key = block_min_u64(key, sh);
    if (threadIdx.x == 0) part[tile] = key;
  }
};

// One LSQR step's rotation and scalars (Sec. IV-A, Paige and Saunders'
// recurrences) from beta^2 and alpha^2; sc = {1 / alpha (v scale), 1 / rho,
// phi, theta / rho, c}.  One thread.
__device__ inline void lsqr_scalars(LsqrState* s, double b2, double a2, double* sc) {
  const double beta = sqrt(b2);
  const double alpha = sqrt(a2);
  const double alpha_old = s->alpha;
  s->anorm2 += alpha_old * alpha_old + beta * beta;
  const double rho = hypot(s->rhobar, beta);
  const double c = s->rhobar / rho, sn = beta / rho;
  const double theta = sn * alpha;
  s->rhobar = -c * alpha;
  const double phi = c * s->phibar;
  s->phibar = sn * s->phibar;
  s->alpha = alpha;
  s->beta = beta;
  sc[0] = alpha > 0.0 ? 1.0 / alpha : 0.0;
  sc[1] = 1.0 / rho;
  sc[2] = phi;
  sc[3] = theta / rho;
  sc[4] = c;
}

// The step's estimates and stopping rule from ||d_k||^2 and ||x||^2.  One thread.
__device__ inline void lsqr_close(LsqrState* s, double dd, double xx, double c) {
  s->ddnorm += dd;
  s->rnorm = s->phibar;
  s->arnorm = s->phibar * s->alpha * fabs(c);
  s->anorm = sqrt(s->anorm2);
  s->acond = s->anorm * sqrt(s->ddnorm);
  s->xnorm = sqrt(xx);
  s->itn += 1;
  int istop = 0;
  if (s->rnorm <= s->btol * s->bnorm + s->atol * s->anorm * s->xnorm) istop = 1;
  else if (s->arnorm <= s->atol * s->anorm * s->rnorm) istop = 2;
  else if (s->acond >= s->conlim) istop = 3;
  else if (s->alpha == 0.0 || s->beta == 0.0) istop = 4;
  else if (s->itn >= s->itnlim) istop = 7;
  s->istop = istop;
  s->done = istop != 0;
}

// The vector part of a step for entry k: v scaled, x += phi w / rho,
// w = v - (theta / rho) w; adds |d_k|^2 and x_k^2 to dd and xx.
__device__ inline void lsqr_vectors(const double* sc, float vraw, float wold, float xold, float* v, float* w, float* x,
                                    int k, double& dd, double& xx) {
  const double vk = (double)vraw * sc[0];
  const double wk = (double)wold;
  const double dk = wk * sc[1];
  dd += dk * dk;
  const float xk = (float)((double)xold + sc[2] * dk);
  x[k] = xk;
  xx += (double)xk * xk;
  const float vf = (float)vk;
  v[k] = vf;
  w[k] = (float)((double)vf - sc[3] * wk);
}

// LSQR: v <- Psi_F^H u / beta - beta v   (or Psi_F^H u / beta at the start),
// with u held unnormalised; per-tile partial sums of v^2.  With ls set (the
// whole list in one workgroup, not the first step) the workgroup also takes
// the step of lsqr_update_kernel: the same sums in the same order, so the
// iterates are those of the separate launch.
struct EpiLsqrV {
  float* v;
  const double* beta_part;
  int nbeta;
  double* alpha_part;
  int first;
  LsqrState* ls = nullptr;
  float* w = nullptr;
  float* x = nullptr;
  using Ctx = NoCtx;
  struct Pre {
    float v, w, x;  // the column's old v, w and x
  };
  __device__ Ctx init() const { return {}; }
  __device__ Pre prefetch(int col, bool ok) const {
    Pre p{0.f, 0.f, 0.f};
    if (ok) {
      if (!first) p.v = v[col];
      if (ls) {
        p.w = w[col];
        p.x = x[col];
      }
    }
    return p;
  }
  __device__ void operator()(int tile, int col, int, float g, bool ok, const Ctx&, const Pre& pf) const {
    __shared__ double sh[8];
    __shared__ double sbeta, sb2;
    __shared__ double sc[5];
    if (threadIdx.x < 64) {  // wave 0, the same order as the LSQR scalar kernels
      const double s = wave_sum_parts(beta_part, nbeta);
      if (threadIdx.x == 0) {
        sb2 = s;
        sbeta = sqrt(s);
      }
    }
    __syncthreads();
    const double beta = sbeta;
    double vr2 = 0.0;
    float vf = 0.f;
    if (ok) {
      double vr = beta > 0.0 ? (double)g / beta : 0.0;
      if (!first) vr -= beta * (double)pf.v;
      vf = (float)vr;
      v[col] = vf;
      vr2 = (double)vf * vf;
    }
    const double tot = block_sum_dpp_d(vr2, sh);
    if (!ls) {
      if (threadIdx.x == 0) alpha_part[tile] = tot;
      return;
    }
    if (threadIdx.x == 0) {
      alpha_part[tile] = tot;
      lsqr_scalars(ls, sb2, tot, sc);
    }
    __syncthreads();
    double dd = 0.0, xx = 0.0;
    if (ok) lsqr_vectors(sc, vf, pf.w, pf.x, v, w, x, col, dd, xx);
    dd = block_sum_dpp_d(dd, sh);
    xx = block_sum_dpp_d(xx, sh);
    if (threadIdx.x == 0) lsqr_close(ls, dd, xx, sc[4]);
  }
};

// LSQR (fused form): v_raw <- Psi_F^H u / beta - beta v_it (or Psi_F^H u / beta
// at the start); beta from the per-wave partials of the correlation kernel.
struct EpiLsqrV2 {
  float* vraw;
  const float* vnorm;
  const double* beta_part;
  int nbeta;
  double* alpha_part;
  int first;
  struct Ctx {
    double beta;
  };
  struct Pre {
    float v;
  };
  // beta_{it+1} from the correlation's per-wave partials, once per block
  // (LDS slots for up to 16 waves: also run by the 12-wave list kernel)
  __device__ Ctx init() const {
    __shared__ double sh[16];
    double b2 = 0.0;
    for (int i = threadIdx.x; i < nbeta; i += blockDim.x) b2 += beta_part[i];
    return {sqrt(block_sum_d(b2, sh))};
  }
  __device__ Pre prefetch(int col, bool ok) const { return {(ok && !first) ? vnorm[col] : 0.f}; }
  __device__ void operator()(int tile, int col, int, float g, bool ok, const Ctx& cx,
                             const Pre& pf) const {
    __shared__ double sh2[16];
    const double beta = cx.beta;
    double vr2 = 0.0;
    if (ok) {
      double vr = beta > 0.0 ? (double)g / beta : 0.0;
      if (!first) vr -= beta * (double)pf.v;
      const float vf = (float)vr;
      vraw[col] = vf;
      vr2 = (double)vf * vf;
    }
    const double tot = block_sum_d(vr2, sh2);
    if (threadIdx.x == 0) alpha_part[tile] = tot;
  }
};

struct LsqrPersistParams {
  int MT, P, n, ntp;
  const float* xf;     // steering vectors of the free set (xf_kernel layout)
  const float2* B;     // right-hand side b (P x P)
  float* frag;         // Ut fragments of u, exchanged between workgroups
  double* pbeta;       // per-workgroup ||u||^2 partials
  double* palpha;      // per-workgroup ||v_raw||^2 partials
  float* vraw;         // v_raw of every free pixel
  float* x_out;        // final iterate
  LsqrState* Sfinal;   // final state
  int* done;           // set when x_out and Sfinal are written
  unsigned* bar;       // grid-barrier counter (zeroed before the launch)
  int* err;            // set if a grid barrier does not complete
  double atol, btol, conlim;
  int itnlim;
};

struct LsqrCuParams {
  int P, n;
  const float* xf;     // steering vectors of the free set (xf_kernel layout)
  const float2* B;     // right-hand side b (P x P, Hermitian)
  float* x_out;        // final iterate
  LsqrState* Sfinal;   // final state
  int* done;           // set when x_out and Sfinal are written
  double atol, btol, conlim;
  int itnlim;
};

struct CorrOsParams {
  int MT, P;
  const float* xf;   // steering vectors of the free set (xf_kernel layout)
  int n;
  const float* vals; // weight of term k: vals[gidx ? gidx[k] : k]
  const int* gidx;
  float2* out;
  const float2* B;
  float cK, cB;
  float* frag;
  const int* stop_flag;
};

// ---- launchers (ops.hip) ----
int adjoint_tile_width(int MT);
hipError_t launch_adjoint_store(const AdjParams& pr, float* out, float scale, hipStream_t st);
hipError_t launch_adjoint_mf(const AdjParams& pr, float* mf, float* eps, float eps_scale,
                             hipStream_t st);
hipError_t launch_adjoint_mvdr(const AdjParams& pr, float* gamma, double C, double kb_coef,
                               hipStream_t st);
hipError_t launch_adjoint_lambda(const AdjParams& pr, const uint8_t* state, uint64_t* part,
                                 hipStream_t st);
hipError_t launch_adjoint_lsqr(const AdjParams& pr, float* v, const double* beta_part, int nbeta,
                               double* alpha_part, int init, hipStream_t st);
// The step of lsqr_update_kernel folded into the adjoint's epilogue: the list
// must fit one epilogue workgroup (adjoint_lsqr_fuses); v, w, x as there
bool adjoint_lsqr_fuses(const AdjParams& pr);
hipError_t launch_adjoint_lsqr_step(const AdjParams& pr, float* v, const double* beta_part, int nbeta,
                                    double* alpha_part, LsqrState* ls, float* w, float* x, hipStream_t st);
hipError_t launch_adjoint_lsqr2(const AdjParams& pr, const EpiLsqrV2& epi, hipStream_t st);
// the column dots of each of pr.nblk blocks apart: out[k * stride + col], one block per workgroup row
hipError_t launch_adjoint_store_blocks(const AdjParams& pr, float* out, size_t stride, hipStream_t st);
int adjoint_lsqr2_tile_width(int MT, int n);
// optional device timestamps of a launch sequence (hipExtLaunchKernel): the
// start of its first kernel goes to `start`, the end of its last kernel to
// `stop`; null events record nothing
struct Stamps {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
// beam.hip (register-resident full-grid beamformer, P <= 48)
bool beam_fits(int P);
int beam_grid(int Q);  // workgroups of a full-grid launch (= partial keys of the lambda variant)
// workgroups of one request in a batched multiplier launch when each wave
// walks `tiles` 16-pixel tiles: the fragments a workgroup builds then serve
// more MFMAs, while the batch still has workgroups enough for the chip
int beam_grid_batched(int Q, int tiles);
// tiles per wave for n requests of Q pixels: the largest power of two up to 16
// that leaves the launch at least 1024 workgroups (1 for small batches)
int beam_batch_tiles(int n, int Q);
hipError_t launch_beam_prep(const float2* U, int P, float* frag, hipStream_t st, Stamps ts = {});
// the fragments come from frag (beam_prep layout) when U is null, else are built from U
hipError_t launch_beam_mf(const float* frag, const float2* U, int P, const Tables& tab, float* mf, float* eps,
                          float eps_scale, hipStream_t st, Stamps ts = {});
hipError_t launch_beam_mvdr(const float* frag, const float2* U, int P, const Tables& tab, float* gamma, double C,
                            double kb_coef, hipStream_t st);
hipError_t launch_beam_store(const float* frag, const float2* U, int P, const Tables& tab, float* out,
                             float scale, hipStream_t st);
// scale (may be null): per-pixel positive factor applied to g before the multiplier
hipError_t launch_beam_lambda(const float* frag, const float2* U, int P, const Tables& tab, const int* skip,
                              const uint8_t* state, uint64_t* part, const float* scale, hipStream_t st);
// one request of a batched multiplier launch
struct BeamLamItem {
  const float2* U;  // gradient matrix E (P x P)
  Tables tab;
  const int* skip;
  const uint8_t* state;
  uint64_t* part;      // nblk argmin keys
  const float* scale;  // optional per-pixel factor
  int P;
  int nblk;  // this request's blocks (beam_grid of its Q); blocks beyond it exit at once
};
// grid: nreq x bpr blocks, bpr >= every item's nblk; all items share P's tile count
hipError_t launch_beam_lambda_batch(const BeamLamItem* items, int nreq, int bpr, int P, hipStream_t st);
// Set-up beamformers of a batch of requests in one launch (P <= 48): grid.y 0
// gives each request's dirty image a^H R a and detection thresholds, grid.y 1
// its MVDR bound from R^-1.  Per pixel the same arithmetic as the full-grid
// launches, so each result is bit-identical to the request's own set-up.
struct BeamSetItem {
  const float2* R;
  const float2* Rinv;
  Tables tab;
  float* mf;
  float* eps;
  float* gamma;
  float eps_scale;
  double C, kb;  // MVDR bound C / h + kb / h
  int P;
  int nblk;
};
hipError_t launch_beam_setup_batch(const BeamSetItem* items, int nreq, int bpr, int P, hipStream_t st);

// GEMM-shaped full-grid beamformer for larger arrays (P <= 288)
bool beam_big_fits(int P);
size_t beam_big_frag_floats(int P);
// workgroups (= partial keys of the lambda variant) with nt 16-pixel tiles per
// workgroup (2, 4, or 8 up to P = 192; anything else: the default for P); nt = 2
// gives the largest grid
int beam_big_grid(int P, int Q, int nt = 0);
constexpr int kBigTileChoices[3] = {2, 4, 8};
// tile counts built for rpw row tiles per wave: 2, 4, and 8 up to rpw 6
// (FP32) or 4 (split half precision, whose block operands stay in LDS)
bool beam_tiles_offered(bool half, int nt, int rpw);
hipError_t launch_beam_prep_full(const float2* U, int P, float* frag, hipStream_t st, Stamps ts = {});
// kind: 0 MF (+ threshold), 1 MVDR bound, 2 store (scaled), 3 multipliers with argmin keys
// lam_scale (kind 3, optional): positive per-pixel factor of the multipliers (PWLS: 1 / D_i)
hipError_t launch_beam_big(int kind, const float* frag, const Tables& tab, const int* skip, float* out, float* eps,
                           float eps_scale, double C, double kb, float scale, const uint8_t* state, uint64_t* part,
                           hipStream_t st, Stamps ts = {}, int nt = 0, const float* lam_scale = nullptr);
// the FP16 scale buffer (`scale` below): the scale, then the partial maxima it is formed from
constexpr int kHalfScaleParts = 64;
constexpr int kHalfScaleFloats = 1 + kHalfScaleParts;
// the same full-grid products in split half precision (FP16 with power-of-two
// scaling, or BF16): fragments and scale (kHalfScaleFloats floats) prepared by
// launch_beam_prep_h16
int beam_h16_chunks(int P);
size_t beam_h16_frag_bytes(int P);
hipError_t launch_beam_prep_h16(const float2* U, int P, bool bf16, void* frag, float* scale, hipStream_t st,
                                Stamps ts = {});
hipError_t launch_beam_h16(int kind, bool bf16, const void* frag, const float* scale, const Tables& tab,
                           const int* skip, float* out, float* eps, float eps_scale, double C, double kb, float sc,
                           const uint8_t* state, uint64_t* part, hipStream_t st, Stamps ts = {}, int nt = 0);
// sums over covariance blocks of the full-grid beamformer (any P, any precision:
// prec 0 FP32, 1 FP16 split, 2 BF16 split); frag_big / frag_half / hscale are
// the scratch of the GEMM-shaped and half-precision kernels
// Reduced precision with FP32 refinement (host-driven loop, CLSIMG_FP16 /
// CLSIMG_BF16): approximate multipliers of every pixel from one half-precision
// product of the block-triangular Ut of E (lam[] and one argmin key per
// workgroup in keys[]), then the pixels within twice the rounding bound of
// the approximate minimum are listed in cand[] (*count of them, possibly more
// than cap) for an FP32 evaluation.  frag: beam_h1_frag_bytes(P); scale:
// kHalfScaleFloats floats (FP16); absum: nabs doubles; keys: beam_big_grid(P, Q, nt) entries.
size_t beam_h1_frag_bytes(int P);
double beam_h1_delta_coef(int P, bool bf16);
hipError_t launch_beam_lambda_refined(const float2* E, int P, bool bf16, const Tables& tab, const int* skip,
                                      const uint8_t* state, void* frag, float* scale, double* absum, int nabs,
                                      uint64_t* keys, float* lam, int* cand, int cap, int* count, hipStream_t st,
                                      int nt, Stamps ts = {});
hipError_t launch_beam_accumulate(const float2* U, int P, const Tables& tab, const int* skip, float* sum,
                                  float* sumsq, float scale, int first, int prec, float* frag_big, void* frag_half,
                                  float* hscale, hipStream_t st, int nt = 0);
// K covariance blocks: images, bound and multipliers from the block sums
hipError_t launch_multi_mf(const float* mfsq, int Q, float eps_coef, float* eps, hipStream_t st);
hipError_t launch_multi_bound(int kind, const float* s1, const float* s2, int Q, double C, double K, double kb_coef,
                              float* gamma, hipStream_t st);
int lambda_vec_blocks(int Q);
hipError_t launch_lambda_vec(const float* g, const uint8_t* state, int Q, const int* skip, uint64_t* part,
                             hipStream_t st);
// offgrid.hip: strong off-grid correction of the free pixels (Sec. III-E)
hipError_t launch_xf_off(const double* pos, int P, double lam, int nl, double l0, double dl, double m0, double dm,
                         const int* Flist, int n, const float* delta, float* xf, hipStream_t st);
hipError_t launch_newton_offset(const float2* E, int P, const double* pos, double lam, const int* Flist, int n,
                                const float* z, const float* xf, float* delta, float half_l, float half_m,
                                hipStream_t st);
hipError_t launch_gamma_off(int kind, const float2* M, int P, const int* Flist, int n, const float* xf, double C,
                            double kb, float* gamma, hipStream_t st);
hipError_t launch_offgrid_sets(const uint8_t* state, int Q, const float* gamma0, float* delta, float* sigma,
                               hipStream_t st);
hipError_t launch_frob2(const float2* M, int n, double* out, hipStream_t st);
// lsqr_cu.hip
bool lsqr_cu_fits(int P, int n);
hipError_t launch_lsqr_cu(const LsqrCuParams& pr, hipStream_t st);
// lsqr_persist.hip
bool persist_fits(int P, int n);
int persist_grid(int P, int n);
hipError_t launch_lsqr_persist(const LsqrPersistParams& pr, hipStream_t st);
// lsqr.hip
int lsqr_fwd_waves(int P);
hipError_t launch_corr_os(const CorrOsParams& pr, hipStream_t st);
hipError_t launch_xf(const Tables& tab, const int* Flist, int n, float* xf, hipStream_t st);
hipError_t launch_lsqr_fwd(const LsqrFwdParams& pr, hipStream_t st);
// x0 <- x1 when the finished two-kernel LSQR (state S) ended on an odd step
hipError_t launch_lsqr_pick(const LsqrState* S, const float* x1, float* x0, int n, hipStream_t st);
hipError_t launch_lsqr_setup(LsqrState* S0, int* done, double atol, double btol, double conlim,
                             int itnlim, hipStream_t st);
void forward_plan(int P, int n, int* chw, int* nchunks);
int forward_chunks_max(int P);       // most chunks (partials per block pair) of the correlation
size_t forward_part_floats(int P);   // floats of one chunk's partials
hipError_t launch_forward(const FwdParams& pr, hipStream_t st);
int reduce_blocks(int P);
hipError_t launch_reduce(const RedParams& pr, hipStream_t st);
// a short list (corr_small_fits) in one launch: the output of launch_forward
// followed by launch_reduce, without the partial tiles (f.part unused)
bool corr_small_fits(int n, int nblk);
hipError_t launch_corr_small(const FwdParams& f, const RedParams& pr, hipStream_t st);
// W: chol_work_elems(P) FP64 complex entries (unused for P <= kCholLdsMaxP)
size_t chol_work_elems(int P);
hipError_t launch_chol_inverse(const float2* R, int P, double2* W, double2* Li, float2* Rinv,
                               int* status, hipStream_t st);
// one covariance of a batched factorisation (P <= kCholLdsMaxP, LDS-resident)
constexpr int kCholLdsMaxP = 64;
struct CholItem {
  const float2* R;  // P x P complex64
  double2* Li;      // L^-1 (P x P, FP64) or null
  float2* Rinv;     // R^-1 as complex64
  int* status;      // 0 ok, 1 not positive definite, 2 non-finite entry
};
// items: DEVICE array of n; one workgroup each
hipError_t launch_chol_inverse_batch(const CholItem* items, int n, int P, hipStream_t st);
// antenna-fastest copies ElT (nl x corr_rows(Pp)), EmT (nm x corr_rows(Pp)) of the tables, zero beyond Pp
hipError_t launch_tables_t(const float2* El, const float2* Em, int Pp, int nl, int nm, float2* ElT, float2* EmT,
                           hipStream_t st);
hipError_t launch_tables(const double* pos, int P, double lambda, int nl, int nm, double l0,
                         double dl, double m0, double dm, float2* El, float2* Em, hipStream_t st);
// Steering tables of a batch of geometries in one launch, every entry as
// launch_tables computes it.  total_max: the largest Pp (nl + nm).
struct TableItem {
  const double* pos;  // 2P positions (x, y), device
  double lambda, l0, dl, m0, dm;
  int P, nl, nm;
  float2* El;
  float2* Em;
};
hipError_t launch_tables_batch(const TableItem* items, int nreq, int total_max, hipStream_t st);
hipError_t launch_sub_diag(const float2* R, const float* noise, int P, float2* B0, hipStream_t st);
hipError_t launch_fill(float* x, float v, int n, hipStream_t st);

// ---- active-set / LSQR control kernels (solve.hip) ----
struct SolveDecision {
  int lsqr_done, lsqr_itn, lsqr_istop;
  int feasible;          // subproblem solution inside the box
  int ib, ib_to;         // blocking pixel and its new state (infeasible step)
  float mu_max;
  float margin_z;        // min over F of min(z, gamma - z)/gamma (feasible only)
  int nF, nU;            // set sizes after the step
  int i_min;             // most negative multiplier (feasible only; -1: none)
  int st_min;            // set of i_min (0 = L, 2 = U)
  float lam_min, eps_min;
  int grad_done;
  int lsqr_err;          // a grid barrier of the LSQR kernel did not complete
  int cand_overflow;     // refined multipliers: more candidates than the list holds
};

// sorted lists of F and U and their sizes (dec->nF, dec->nU); part: compact_parts(Q) ints
int compact_parts(int Q);
hipError_t launch_compact(const uint8_t* state, int Q, int* Flist, int* Ulist, SolveDecision* dec, int* part,
                          hipStream_t st);

// ---- device-resident outer iteration (outer.hip) ----
// pixel states and stop codes as in the public header
constexpr int kStateL = 0, kStateF = 1, kStateU = 2;
constexpr int kStatusMaxOuter = 1, kStatusCycle = 3;

struct OuterState {
  int done;          // the iteration has stopped (or handed over: fallback)
  int status;        // 0, kStatusMaxOuter or kStatusCycle
  int fallback;      // stopped because the next free set does not fit one workgroup
  int await_lambda;  // a feasible step left E; the multiplier keys decide the next move
  int lam_skip;      // the multiplier kernel has nothing to do
  int nF, nU;
  int ucur;          // which half of the two-buffer U list is current
  int outer, adds, drops, lsqr_total, itnlim_hits, last_added;
  int bb_dirty;      // U changed since b was formed
  int last_itn, last_istop, last_feasible, last_ib, last_ib_to, last_imin;
  float last_mu, last_lam, last_eps;
  double margin_lambda, margin_z, psi_flops;
  double b0n2;  // ||B0||^2 (data of the problem solved: whitened for PWLS)
  double res2;  // ||Psi sigma - b||^2 at the last feasible step
};

struct OuterParams {
  OuterState* st;
  int* Flist;  // sorted free pixels (capacity Q)
  int* Ulist;  // sorted pixels at the upper bound, two buffers of Q entries
  float* sigma;
  const float* gamma;
  const float* eps;
  uint8_t* state;
  const float2* B0;
  float2* Bb;
  float2* E;
  const uint64_t* keys;  // per-block argmin keys of the multiplier kernel
  int nkeys;
  Tables tab;
  int P, Q;
  double atol, btol, conlim;
  int itnlim, max_outer;
  int max_f;  // largest free set kept on the device (at most the LDS capacity)
  // PWLS (eq. preWLS), both null for LS: steering rows are L^-1 a_i * rowscale_i,
  // and the gradient matrix handed to the multiplier kernel is L^-H E L^-1
  const float2* Lw;       // L^-1, P x P row-major (lower triangular)
  const float* rowscale;  // 1 / sqrt(D_i)
};

bool outer_fits(int P);
hipError_t launch_pwls_setup(const float* h, const float* gamma, double C, double kd_coef, int Q, float* rowscale,
                             float* gamma_pw, float* eps_pw, float* dinv, hipStream_t st);
hipError_t launch_pwls_whiten(const double2* Li, const float2* B0, int P, float2* Lw, float2* B0w, hipStream_t st);
hipError_t launch_pwls_scale(float* x, const float* s, int n, bool divide, hipStream_t st);
// out = L^-1 herm(X) L^-H (colour false) or L^-H herm(X) L^-1 (colour true), FP64
// temporary T (P x P); norm2 (optional): per row of out, its squared norm
hipError_t launch_pwls_sandwich(const double2* Li, const float2* X, int P, bool colour, double2* T, float2* out,
                                double* norm2, hipStream_t st);
// xf rows (xf_kernel layout) whitened in place: rowscale[F[k]] L^-1 x_k
hipError_t launch_pwls_xf_whiten(const double2* Li, int P, const int* Flist, int n, const float* rowscale, float* xf,
                                 hipStream_t st);
hipError_t launch_outer_init(OuterState* st, const SolveDecision* dec, hipStream_t s);
// Fresh state of a batch of requests in one launch: B0 = R - diag(noise),
// sigma = 0, every pixel at its lower bound, a fresh outer state.
struct ReqInitItem {
  const float2* R;
  const float* noise;  // optional
  float2* B0;
  float* sigma;
  uint8_t* state;
  OuterState* st;
  int P, Q;
};
hipError_t launch_request_init_batch(const ReqInitItem* items, int nreq, int Qmax, hipStream_t s);
hipError_t launch_outer_step(const OuterParams& pr, hipStream_t s);
// prs: device array of nreq parameter sets with the same P
hipError_t launch_outer_step_batch(const OuterParams* prs, int nreq, int P, hipStream_t s);
// copies every request's outer state (prs[r].st) to out[r] (device)
hipError_t launch_gather_states(const OuterParams* prs, int n, OuterState* out, hipStream_t s);
hipError_t launch_lsqr_init_scalars(LsqrState* s, const double* beta_part, int nbeta,
                                    const double* alpha_part, int nalpha, float* v, float* w,
                                    float* x, int n, double atol, double btol, double conlim,
                                    int itnlim, hipStream_t st);
// v from the per-block adjoint dots (launch_adjoint_store_blocks), 64-column alpha partials
hipError_t launch_lsqr_v_blocks(const float* gpart, int K, size_t stride, int n, float* v, const double* beta_part,
                                int nbeta, double* alpha_part, int first, const int* stop, hipStream_t st);
hipError_t launch_lsqr_update(LsqrState* s, const double* beta_part, int nbeta,
                              const double* alpha_part, int nalpha, float* v, float* w, float* x,
                              int n, hipStream_t st);
hipError_t launch_step(const int* done, const int* err, const LsqrState* s, const float* x0,
                       const float* x1, const int* Flist, int nF, float* sigma, const float* gamma,
                       uint8_t* state, SolveDecision* dec, hipStream_t st);
hipError_t launch_lsqr_setup2(LsqrState* S0, int* done, unsigned* bar, int* err, double atol,
                              double btol, double conlim, int itnlim, hipStream_t st);
hipError_t launch_argmin_final(const uint64_t* part, int nparts, const float* eps,
                               const uint8_t* state, SolveDecision* dec, hipStream_t st,
                               const int* cand_count = nullptr, int cand_cap = 0);
hipError_t launch_set_state(uint8_t* state, int i, uint8_t v, hipStream_t st);
hipError_t launch_init_state(const float* sigma0, const uint8_t* state0, float* sigma,
                             uint8_t* state, int Q, hipStream_t st);

}  // namespace clsimg
