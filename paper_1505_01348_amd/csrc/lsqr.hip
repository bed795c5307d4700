// Free-set kernels of the active-set solve: the steering vectors of the free
// pixels, the output-stationary correlation over them, and the fused LSQR step
// (Sec. IV-A / IV-B).
//
// One LSQR step is two kernels:
//   lsqr_fwd_kernel(it):  finish step it-1 (FP64 rotation scalars, v, w, x and
//                         the stopping tests) and compute
//                         u_{it+1} = Psi_F v_it - (alpha_it/beta_it) u_it
//                         with its Ut fragments and ||u||^2 partials;
//   adjoint_kernel<EpiLsqrV2>(it):
//                         v_raw = Psi_F^H u_{it+1} / beta_{it+1} - beta_{it+1} v_it
//                         with ||v_raw||^2 partials.
// Every workgroup of lsqr_fwd_kernel forms alpha and beta itself from the same
// partials in the same order, so all of them agree bit for bit without a grid
// barrier; workgroup 0 alone completes the rotation, writes the vectors and
// the state and takes the stopping decision, which the following launches
// read from the done flag.  Scalars and vectors whose old and new values are
// both live are double-buffered by iteration parity: x_j lives in x[j & 1],
// w_j in w[j & 1], the state after step j in S[(j + 1) & 1].
//
// The correlation is output-stationary: one wave owns one 16 x 16 tile
// (mt <= nt) of G = X_F diag(v) X_F^T, loads its two 16-row slices of the
// real-embedded steering vectors and the weights straight into registers
// (128 pixels at a time, the first 128 requested at launch), and writes the
// Hermitian mirror of an off-diagonal tile itself.  No LDS, no partial sums,
// no reduction kernel.  The steering vectors of the free set are generated
// once per subproblem (xf_kernel, 2Pp x |F| floats) and read by every LSQR
// step.
#include "os_tiles.h"

namespace clsimg {

// X_F[k][2p + s] = Re/Im a_{Flist[k]}[p]  (pixel-major, 2Pp floats per pixel)
__global__ void xf_kernel(Tables tab, const int* __restrict__ Flist, int n, float* __restrict__ xf) {
  const int Pp = tab.Pp;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * Pp; e += gridDim.x * blockDim.x) {
    const int k = e / Pp, p = e - k * Pp;
    const int pix = Flist[k];
    *reinterpret_cast<float2*>(xf + (size_t)k * 2 * Pp + 2 * p) = tab.a(p, pix % tab.nl, pix / tab.nl);
  }
}

// Operands of one wave's tile for 32 k steps (128 pixels) straight from X_F:
// at step s lane (c16, q) takes pixel k0 + 4 s + q, rows 16 mt + c16 and
// 16 nt + c16 of its real-embedded steering vector, and its weight (zero
// past the list; the pixel index is clamped into it, so every load stays in
// X_F).  n >= 1.
constexpr int kOsSteps = 32;

struct OsOps {
  float a[kOsSteps], b[kOsSteps], v[kOsSteps];
};

__device__ inline void os_load(const float* __restrict__ xf, int n, int Pp, const float* __restrict__ vals,
                               const int* __restrict__ gidx, int k0, int mt, int nt, OsOps& o) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
  // the gathered weights' indices first: a wait for them then leaves the
  // operand loads issued after them in flight
  int wi[kOsSteps];
#pragma unroll
  for (int s = 0; s < kOsSteps; ++s) wi[s] = min(k0 + 4 * s + q, n - 1);
  if (gidx) {
#pragma unroll
    for (int s = 0; s < kOsSteps; ++s) wi[s] = gidx[wi[s]];
  }
#pragma unroll
  for (int s = 0; s < kOsSteps; ++s) {
    const float* row = xf + (size_t)min(k0 + 4 * s + q, n - 1) * 2 * Pp;
    o.a[s] = row[16 * mt + c16];
    o.b[s] = row[16 * nt + c16];
  }
#pragma unroll
  for (int s = 0; s < kOsSteps; ++s) {
    const float w = vals[wi[s]];
    o.v[s] = k0 + 4 * s + q < n ? w : 0.f;
  }
}

__device__ inline void os_mma(const OsOps& o, v4f (&acc)[4]) {
#pragma unroll
  for (int s = 0; s < kOsSteps; ++s) acc[s & 3] = mfma16x16x4(o.a[s] * o.v[s], o.b[s], acc[s & 3]);
}

// The tile sum over the whole list; `o` holds the operands of the first 128
// pixels (loaded by the caller, so that their round trip overlaps the
// caller's other work), later chunks are loaded here one after another.
__device__ inline v4f os_accumulate(const float* __restrict__ xf, int n, int Pp, const float* __restrict__ vals,
                                    const int* __restrict__ gidx, int mt, int nt, OsOps& o) {
  v4f acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
  os_mma(o, acc);
  for (int k0 = 4 * kOsSteps; k0 < n; k0 += 4 * kOsSteps) {
    os_load(xf, n, Pp, vals, gidx, k0, mt, nt, o);
    os_mma(o, acc);
  }
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// out = cK K + cB Bold (Bold preloaded), Ut fragments, sum |out|^2 of the lane.
__device__ inline double os_write(v4f acc, const OsSlots& sl, const float2* Bold, int P, int Pp,
                                  float cK, float cB, float2* out, float* frag) {
  float2 K[4], r[4];
  os_assemble(acc, sl, K);
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = make_float2(cK * K[i].x + cB * Bold[i].x, cK * K[i].y + cB * Bold[i].y);
  return os_store(sl, r, P, Pp, out, frag);
}

// ---------------------------------------------------------------------------
// Each workgroup has five waves.  Wave 0 starts finishing step it-1 (its
// lanes hold the same scalars, wave sums on the VALU): as soon as alpha and
// beta are known it hands 1 / alpha and -alpha / beta to the tile waves
// through one barrier; in workgroup 0 it then completes the rotation, the
// vector updates and the stopping tests while they write.  Waves 1-4 each own one tile of Psi_F v_raw (formed
// before the barrier, scaled by 1 / alpha after it).  The tile waves write u,
// its fragments and norm partials also in the step where the tests stop the
// solve: nothing reads them after that (the next kernels see the flag).
constexpr int kFwdVecPre = 4;  // vector entries per lane of wave 0 loaded at launch (n <= 256)
constexpr int kFwdThreads = 320;

__global__ __launch_bounds__(kFwdThreads) void lsqr_fwd_kernel(LsqrFwdParams pr) {
  __shared__ double sc[2];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c16 = lane & 15, q = lane >> 4;
  const int it = pr.it, n = pr.n;
  const bool first = (it == 1);
  const bool wg0 = (blockIdx.x == 0);
  const int MT = pr.MT, P = pr.P, Pp = 8 * MT;
  const int was_done = *pr.done;
  if (w == 0) {
    LsqrState* Sprev = pr.S + ((it - 1) & 1);
    LsqrState* Scur = pr.S + (it & 1);
    float* x_prev = (it & 1) ? pr.x1 : pr.x0;  // x_{it-2}
    float* x_cur = (it & 1) ? pr.x0 : pr.x1;   // x_{it-1}
    float* w_prev = (it & 1) ? pr.w0 : pr.w1;  // w_{it-1}
    float* w_cur = (it & 1) ? pr.w1 : pr.w0;   // w_it
    // ---- every load first: state, partials, vectors ----
    LsqrState S = *Sprev;  // tolerances and limits travel with the state
    double ap[2] = {0.0, 0.0}, bp[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (lane + 64 * j < pr.nalpha) ap[j] = pr.alpha_part[lane + 64 * j];
      if (lane + 64 * j < pr.nbeta_in) bp[j] = pr.beta_in[lane + 64 * j];
    }
    float vr0[kFwdVecPre], wp0[kFwdVecPre], xp0[kFwdVecPre];
#pragma unroll
    for (int j = 0; j < kFwdVecPre; ++j) {
      const int k = lane + 64 * j;
      vr0[j] = wp0[j] = xp0[j] = 0.f;
      if (k < n) {
        vr0[j] = pr.vraw[k];
        if (!first) {
          wp0[j] = w_prev[k];
          xp0[j] = x_prev[k];
        }
      }
    }
    if (was_done) return;  // uniform: a finished solve
    // ---- finish LSQR step it-1 (every workgroup, identical arithmetic) ----
    double a2 = ap[0] + ap[1], b2 = bp[0] + bp[1];
    for (int i = lane + 128; i < pr.nalpha; i += 64) a2 += pr.alpha_part[i];
    for (int i = lane + 128; i < pr.nbeta_in; i += 64) b2 += pr.beta_in[i];
    a2 = wave_sum_dpp_d(a2);
    b2 = wave_sum_dpp_d(b2);
    const double alpha = sqrt(a2), beta = sqrt(b2);
    const double iv = alpha > 0.0 ? 1.0 / alpha : 0.0;  // v = v_raw / alpha
    if (lane == 0) {
      sc[0] = iv;
      sc[1] = alpha > 0.0 && beta > 0.0 ? -alpha / beta : 0.0;
    }
    __syncthreads();  // the tile waves' scalars
    if (!wg0) return;  // the vectors, the state and the flag are workgroup 0's
    double ir = 0.0, phi = 0.0, tr = 0.0, c = 0.0, sn = 0.0;
    if (!first) {
      const double rho = hypot(S.rhobar, beta);
      c = S.rhobar / rho;
      sn = beta / rho;
      ir = 1.0 / rho;         // d = w / rho
      phi = c * S.phibar;
      tr = sn * alpha / rho;  // theta / rho
    }
    double dd = 0.0, xx = 0.0;
    for (int j = 0, k = lane; k < n; ++j, k += 64) {
      const bool pre = j < kFwdVecPre;
      const float vf = (float)((double)(pre ? vr0[j] : pr.vraw[k]) * iv);
      pr.vnorm[k] = vf;
      if (first) {
        w_cur[k] = vf;
        x_cur[k] = 0.f;
      } else {
        const double wk = (double)(pre ? wp0[j] : w_prev[k]);
        const double dk = wk * ir;
        dd += dk * dk;
        const float xk = (float)((double)(pre ? xp0[j] : x_prev[k]) + phi * dk);
        xx += (double)xk * xk;
        x_cur[k] = xk;
        w_cur[k] = (float)((double)vf - tr * wk);
      }
    }
    dd = wave_sum_dpp_d(dd);
    xx = wave_sum_dpp_d(xx);
    if (first) {
      S.alpha = alpha;
      S.beta = beta;
      S.rhobar = alpha;
      S.phibar = beta;
      S.bnorm = beta;
      S.anorm2 = 0.0;
      S.ddnorm = 0.0;
      S.rnorm = beta;
      S.arnorm = alpha * beta;
      S.anorm = S.acond = S.xnorm = 0.0;
      S.itn = 0;
      S.istop = (n == 0 || alpha == 0.0 || beta == 0.0) ? 4 : 0;
    } else {
      S.anorm2 += S.alpha * S.alpha + beta * beta;
      S.rhobar = -c * alpha;
      S.phibar = sn * S.phibar;
      S.alpha = alpha;
      S.beta = beta;
      S.ddnorm += dd;
      S.rnorm = S.phibar;
      S.arnorm = S.phibar * alpha * fabs(c);
      S.anorm = sqrt(S.anorm2);
      S.acond = S.anorm * sqrt(S.ddnorm);
      S.xnorm = sqrt(xx);
      S.itn = it - 1;
      int istop = 0;
      if (S.rnorm <= S.btol * S.bnorm + S.atol * S.anorm * S.xnorm) istop = 1;
      else if (S.arnorm <= S.atol * S.anorm * S.rnorm) istop = 2;
      else if (S.acond >= S.conlim) istop = 3;
      else if (alpha == 0.0 || beta == 0.0) istop = 4;
      else if (S.itn >= S.itnlim) istop = 7;
      S.istop = istop;
    }
    S.done = S.istop != 0;
    if (lane == 0) {
      *Scur = S;
      if (S.done) {
        // the final iterate x_{itn} stays in x[itn & 1]
        *pr.Sfinal = S;
        *pr.done = 1;
      }
    }
    return;
  }
  // ---- tile waves: u_{it+1} = Psi_F v_it - (alpha/beta) u_it ----
  const int tp = blockIdx.x * 4 + (w - 1);
  const bool active = tp < pr.ntp;
  int mt = 0, nt = 0;
  if (active) tri_tile(tp, MT, mt, nt);
  const OsSlots sl = os_slots(mt, nt, c16, q, P, active);
  float2 uold[4];
  os_prefetch(sl, pr.u, P, uold);
  OsOps ops;
  if (active && n > 0) os_load(pr.xf, n, Pp, pr.vraw, nullptr, 0, mt, nt, ops);
  if (was_done) return;  // uniform: a finished solve
  v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
  if (active) acc = os_accumulate(pr.xf, n, Pp, pr.vraw, nullptr, mt, nt, ops);
  __syncthreads();  // wave 0's scalars
  double nrm = os_write(acc, sl, uold, P, Pp, (float)sc[0], (float)sc[1], pr.u, pr.frag);
  nrm = wave_sum_dpp_d(nrm);
  if (lane == 0) pr.beta_out[tp] = nrm;
}

// Plain output-stationary correlation over the free set:
//   out = cK * sum_k vals[gidx ? gidx[k] : k] a_k a_k^H + cB * B,  Ut fragments of out.
__global__ __launch_bounds__(kThreads) void corr_os_kernel(CorrOsParams pr) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c16 = lane & 15, q = lane >> 4;
  const int MT = pr.MT, P = pr.P, Pp = 8 * MT;
  const int tp = blockIdx.x * 4 + w;
  const bool active = tp < MT * (MT + 1) / 2;
  int mt = 0, nt = 0;
  if (active) tri_tile(tp, MT, mt, nt);
  const OsSlots sl = os_slots(mt, nt, c16, q, P, active);
  const int stop = pr.stop_flag ? *pr.stop_flag : 0;
  float2 bold[4];
  os_prefetch(sl, pr.B, P, bold);
  OsOps ops;
  const bool go = active && pr.n > 0;
  if (go) os_load(pr.xf, pr.n, Pp, pr.vals, pr.gidx, 0, mt, nt, ops);
  if (stop) return;
  v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
  if (go) acc = os_accumulate(pr.xf, pr.n, Pp, pr.vals, pr.gidx, mt, nt, ops);
  (void)os_write(acc, sl, bold, P, Pp, pr.cK, pr.cB, pr.out, pr.frag);
}

__global__ void lsqr_setup_kernel(LsqrState* S0, int* done, double atol, double btol,
                                  double conlim, int itnlim) {
  LsqrState S = {};
  S.atol = atol;
  S.btol = btol;
  S.conlim = conlim;
  S.itnlim = itnlim;
  *S0 = S;
  *done = 0;
}

__global__ void lsqr_setup2_kernel(int* done, unsigned* bar, int* err) {
  *done = 0;
  *bar = 0u;
  *err = 0;
}

hipError_t launch_lsqr_setup2(LsqrState* S0, int* done, unsigned* bar, int* err, double atol,
                              double btol, double conlim, int itnlim, hipStream_t st) {
  (void)S0; (void)atol; (void)btol; (void)conlim; (void)itnlim;
  hipLaunchKernelGGL(lsqr_setup2_kernel, dim3(1), dim3(1), 0, st, done, bar, err);
  return hipGetLastError();
}

hipError_t launch_lsqr_setup(LsqrState* S0, int* done, double atol, double btol, double conlim,
                             int itnlim, hipStream_t st) {
  hipLaunchKernelGGL(lsqr_setup_kernel, dim3(1), dim3(1), 0, st, S0, done, atol, btol, conlim, itnlim);
  return hipGetLastError();
}

// the two-kernel LSQR leaves x_itn in x[itn & 1]: x0 <- x1 when itn is odd
__global__ void lsqr_pick_kernel(const LsqrState* __restrict__ S, const float* __restrict__ x1, float* __restrict__ x0,
                                 int n) {
  if (!(S->itn & 1)) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x0[i] = x1[i];
}

hipError_t launch_lsqr_pick(const LsqrState* S, const float* x1, float* x0, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int g = std::min((n + 255) / 256, 1024);
  hipLaunchKernelGGL(lsqr_pick_kernel, dim3(g), dim3(256), 0, st, S, x1, x0, n);
  return hipGetLastError();
}

int lsqr_fwd_waves(int P) {
  const int MT = pad_p(P) / 8;
  const int ntp = MT * (MT + 1) / 2;
  return 4 * ((ntp + 3) / 4);
}

hipError_t launch_lsqr_fwd(const LsqrFwdParams& pr, hipStream_t st) {
  const int blocks = (pr.ntp + 3) / 4;
  hipLaunchKernelGGL(lsqr_fwd_kernel, dim3(blocks), dim3(kFwdThreads), 0, st, pr);
  return hipGetLastError();
}

hipError_t launch_corr_os(const CorrOsParams& pr, hipStream_t st) {
  const int ntp = pr.MT * (pr.MT + 1) / 2;
  hipLaunchKernelGGL(corr_os_kernel, dim3((ntp + 3) / 4), dim3(kThreads), 0, st, pr);
  return hipGetLastError();
}

hipError_t launch_xf(const Tables& tab, const int* Flist, int n, float* xf, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int grid = (n * tab.Pp + kThreads - 1) / kThreads;
  if (grid > 2048) grid = 2048;
  hipLaunchKernelGGL(xf_kernel, dim3(grid), dim3(kThreads), 0, st, tab, Flist, n, xf);
  return hipGetLastError();
}

}  // namespace clsimg
