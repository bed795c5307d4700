// One LSQR solve of the free-set subproblem in a single cooperative kernel
// (Sec. IV-A, eqs. initbeta, initu, lanczos, with the LSQR updates).
//
// A handful of workgroups (one per four 16 x 16 output tiles of the
// correlation) stay resident for the whole solve.  Each keeps in LDS the
// real-embedded steering vectors of every free pixel, its own copy of the
// LSQR vectors v, w, x, and each lane keeps the elements of u it owns in
// registers.  One LSQR step is:
//   F  correlation tiles: u <- Psi_F v - (alpha/beta) u, Ut fragments and
//      ||u||^2 partials to global memory;             grid barrier
//   A  beamforming of this workgroup's 32 free pixels with the fragments:
//      v_raw = Psi_F^H u / beta - beta v, ||v_raw||^2 partials; grid barrier
//   S  every workgroup reads all of v_raw and the partials and evaluates the
//      FP64 rotation, the vector updates and the stopping tests itself (same
//      inputs, same order: every workgroup takes the same decision).
// The first pass sets u = b instead of running the correlation.  Grid
// barriers are a monotone counter with a bounded spin: a barrier that does not
// complete sets an error flag instead of waiting forever, and every workgroup
// then leaves.
#include "os_tiles.h"

namespace clsimg {

constexpr int kPersistLds = 36864;  // floats of LDS per workgroup (144 KiB)
constexpr long kSpinLimit = 1L << 22;

// row stride of the resident X_F: 2Pp rounded so that stride % 32 == 18,
// which keeps both access patterns (pixel-major rows read by the correlation
// and columns read by the beamforming) nearly free of bank conflicts
__host__ __device__ inline int persist_row_stride(int Pp) {
  const int rs = 2 * Pp;
  return rs + ((18 - rs % 32) + 32) % 32;
}

__host__ __device__ inline int persist_lds_floats(int Pp, int MTA, int n) {
  const int n16 = (n + 15) & ~15;
  return n16 * persist_row_stride(Pp) + MTA * (Pp / 2) * 64 + 4 * n16;
}

__device__ inline bool grid_barrier(unsigned* bar, unsigned target, int* err, int* s_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    __threadfence();
    atomicAdd(bar, 1u);
    long spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) || ++spins > kSpinLimit) {
        atomicExch(err, 1);
        ok = 0;
        break;
      }
    }
    __threadfence();
    *s_flag = ok;
  }
  __syncthreads();
  return *s_flag != 0;
}

template <int MTH>
__global__ __launch_bounds__(kThreads) void lsqr_persist_kernel(LsqrPersistParams pr) {
  constexpr int MTA = 2 * MTH;  // row tiles held for the beamforming (zero padded)
  __shared__ float lds[kPersistLds];
  __shared__ double red[4];
  __shared__ double sc[8];
  __shared__ float gsh[2][32];
  __shared__ int s_flag, s_done;
  __shared__ LsqrState sS;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c16 = lane & 15, q = lane >> 4;
  const int MT = pr.MT, P = pr.P, Pp = 8 * MT, KS = Pp / 2, n = pr.n;
  const int n16 = (n + 15) & ~15;
  const int RS = persist_row_stride(Pp);
  const unsigned G = gridDim.x;
  float* xr = lds;                    // n16 x RS: X_F, pixel-major
  float* fr = xr + n16 * RS;          // MTA x KS x 64: Ut fragments
  float* vv = fr + MTA * KS * 64;     // v_i
  float* ww = vv + n16;               // w_i
  float* xv = ww + n16;               // x_i
  float* vr = xv + n16;               // v_raw of all pixels
  unsigned bar_k = 0;

  // resident steering vectors of the free set (zero rows past n) and zeroed
  // vectors (the padding entries past n must stay zero: they weight zero rows)
  for (int e = tid; e < n16 * 2 * Pp; e += kThreads) {
    const int k = e / (2 * Pp), r = e - k * 2 * Pp;
    xr[k * RS + r] = k < n ? pr.xf[(size_t)k * 2 * Pp + r] : 0.f;
  }
  for (int e = tid; e < 4 * n16; e += kThreads) vv[e] = 0.f;
  // correlation tile of this wave and the u elements it owns
  const int tp = blockIdx.x * 4 + w;
  const bool active = tp < pr.ntp;
  int mt = 0, nt = 0;
  if (active) tri_tile(tp, MT, mt, nt);
  const OsSlots sl = os_slots(mt, nt, c16, q, P, active);
  float2 uown[4];
  os_prefetch(sl, pr.B, P, uown);  // u_1 = b
  // beamforming columns of this workgroup
  const int nt_l = w & 1, mh = w >> 1;
  const int col = blockIdx.x * 32 + 16 * nt_l + c16;
  const bool cvalid = col < n;
  if (tid == 0) {
    LsqrState S = {};
    S.atol = pr.atol;
    S.btol = pr.btol;
    S.conlim = pr.conlim;
    S.itnlim = pr.itnlim;
    sS = S;
  }
  float cu = 0.f;  // -alpha_i / beta_i
  bool first = true, ok = true;
  for (int it = 0;; ++it) {
    // ---- F: u <- Psi_F v - (alpha/beta) u  (or u = b on the first pass) ----
    if (!first) {
      const v4f acc = os_accumulate_lds(xr, vv, n16, RS, active, mt, nt);
      float2 K[4];
      os_assemble(acc, sl, K);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        uown[i].x = K[i].x + cu * uown[i].x;
        uown[i].y = K[i].y + cu * uown[i].y;
      }
    }
    {
      double nb = os_store(sl, uown, P, Pp, nullptr, pr.frag);
      nb = block_sum_d(nb, red);
      if (tid == 0) pr.pbeta[blockIdx.x] = nb;
    }
    if (!(ok = grid_barrier(pr.bar, (++bar_k) * G, pr.err, &s_flag))) break;

    // ---- A: v_raw = Psi_F^H u / beta - beta v on this workgroup's pixels ----
    if (w == 0) {  // all G partials in flight at once, fixed-order wave sum
      const double s = wave_sum_d(lane < (int)G ? pr.pbeta[lane] : 0.0);
      if (lane == 0) sc[0] = sqrt(s);
    }
    for (int e = tid; e < MTA * KS * 16; e += kThreads) {
      const int m = e / (KS * 16);
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (m < MT) v = *reinterpret_cast<const float4*>(pr.frag + 4 * e);
      *reinterpret_cast<float4*>(fr + 4 * e) = v;
    }
    __syncthreads();
    const double beta = sc[0];
    {
      v4f acc[MTH];
#pragma unroll
      for (int mi = 0; mi < MTH; ++mi) acc[mi] = v4f{0.f, 0.f, 0.f, 0.f};
      if (blockIdx.x * 32 < n) {
        for (int kc = 0; kc < KS; ++kc) {
          const float b = cvalid ? xr[col * RS + 4 * kc + q] : 0.f;
#pragma unroll
          for (int mi = 0; mi < MTH; ++mi)
            acc[mi] = mfma16x16x4(fr[((mh * MTH + mi) * KS + kc) * 64 + lane], b, acc[mi]);
        }
      }
      float gp = 0.f;
#pragma unroll
      for (int mi = 0; mi < MTH; ++mi) {
        const int m = mh * MTH + mi;
        if (m < MT && cvalid) {
          const float* xrow = xr + col * RS + 16 * m + 4 * q;
          gp += xrow[0] * acc[mi][0] + xrow[1] * acc[mi][1] + xrow[2] * acc[mi][2] + xrow[3] * acc[mi][3];
        }
      }
      gp += __shfl_xor(gp, 16, 64);
      gp += __shfl_xor(gp, 32, 64);
      if (q == 0) gsh[mh][16 * nt_l + c16] = gp;
    }
    __syncthreads();
    {
      double a2 = 0.0;
      if (tid < 32) {
        const int c = blockIdx.x * 32 + tid;
        if (c < n) {
          double v = beta > 0.0 ? (double)(gsh[0][tid] + gsh[1][tid]) / beta : 0.0;
          if (!first) v -= beta * (double)vv[c];
          const float vf = (float)v;
          pr.vraw[c] = vf;
          a2 = (double)vf * vf;
        }
      }
      a2 = block_sum_d(a2, red);
      if (tid == 0) pr.palpha[blockIdx.x] = a2;
    }
    if (!(ok = grid_barrier(pr.bar, (++bar_k) * G, pr.err, &s_flag))) break;

    // ---- S: rotation, vector updates and stopping tests (every workgroup) ----
    for (int k = tid; k < n; k += kThreads) vr[k] = pr.vraw[k];
    double sa = 0.0;
    if (w == 0) sa = wave_sum_d(lane < (int)G ? pr.palpha[lane] : 0.0);
    if (tid == 0) {
      const double alpha = sqrt(sa);
      sc[1] = alpha;
      sc[2] = alpha > 0.0 ? 1.0 / alpha : 0.0;
      if (!first) {
        const double rho = hypot(sS.rhobar, beta);
        const double c = sS.rhobar / rho, sn = beta / rho;
        sc[3] = 1.0 / rho;         // d = w / rho
        sc[4] = c * sS.phibar;     // phi
        sc[5] = sn * alpha / rho;  // theta / rho
        sc[6] = c;
        sc[7] = sn;
      }
    }
    __syncthreads();
    const double alpha = sc[1], iv = sc[2];
    double dd = 0.0, xx = 0.0;
    if (first) {
      for (int k = tid; k < n; k += kThreads) {
        const float vf = (float)((double)vr[k] * iv);
        vv[k] = vf;
        ww[k] = vf;
        xv[k] = 0.f;
      }
    } else {
      const double ir = sc[3], phi = sc[4], tr = sc[5];
      for (int k = tid; k < n; k += kThreads) {
        const float vf = (float)((double)vr[k] * iv);
        const double wk = (double)ww[k];
        const double dk = wk * ir;
        dd += dk * dk;
        const float xk = (float)((double)xv[k] + phi * dk);
        xx += (double)xk * xk;
        vv[k] = vf;
        xv[k] = xk;
        ww[k] = (float)((double)vf - tr * wk);
      }
    }
    dd = block_sum_d(dd, red);
    xx = block_sum_d(xx, red);
    if (tid == 0) {
      LsqrState S = sS;
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
        S.itn = 0;
        S.istop = (alpha == 0.0 || beta == 0.0) ? 4 : 0;
      } else {
        const double c = sc[6], sn = sc[7];
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
        S.itn = it;
        int istop = 0;
        if (S.rnorm <= S.btol * S.bnorm + S.atol * S.anorm * S.xnorm) istop = 1;
        else if (S.arnorm <= S.atol * S.anorm * S.rnorm) istop = 2;
        else if (S.acond >= S.conlim) istop = 3;
        else if (alpha == 0.0 || beta == 0.0) istop = 4;
        else if (S.itn >= S.itnlim) istop = 7;
        S.istop = istop;
      }
      S.done = S.istop != 0;
      sS = S;
      s_done = S.done;
    }
    __syncthreads();
    if (s_done) break;
    cu = (float)(-alpha / beta);
    first = false;
  }
  // workgroup 0 publishes the result: x_itn, the final state, the flag
  if (blockIdx.x == 0 && ok) {
    for (int k = tid; k < n; k += kThreads) pr.x_out[k] = xv[k];
    __syncthreads();
    if (tid == 0) {
      *pr.Sfinal = sS;
      __threadfence();
      *pr.done = 1;
    }
  }
}

int persist_mth(int MT) { return MT <= 4 ? 2 : (MT <= 8 ? 4 : 0); }

int persist_grid(int P, int n);

// the partial sums are read by one wave: at most 64 workgroups
bool persist_fits(int P, int n) {
  const int MT = pad_p(P) / 8;
  const int mth = persist_mth(MT);
  if (!mth || n <= 0 || persist_grid(P, n) > 64) return false;
  return persist_lds_floats(8 * MT, 2 * mth, n) <= kPersistLds;
}

int persist_grid(int P, int n) {
  const int MT = pad_p(P) / 8;
  const int ntp = MT * (MT + 1) / 2;
  const int a = (ntp + 3) / 4, b = (n + 31) / 32;
  return a > b ? a : b;
}

hipError_t launch_lsqr_persist(const LsqrPersistParams& pr, hipStream_t st) {
  const int G = persist_grid(pr.P, pr.n);
  LsqrPersistParams p = pr;
  void* args[] = {&p};
  const void* fn = persist_mth(pr.MT) == 2 ? reinterpret_cast<const void*>(&lsqr_persist_kernel<2>)
                                           : reinterpret_cast<const void*>(&lsqr_persist_kernel<4>);
  return hipLaunchCooperativeKernel(fn, dim3(G), dim3(kThreads), args, 0, st);
}

}  // namespace clsimg
