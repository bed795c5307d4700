// One LSQR solve of the free-set subproblem on one compute unit (Sec. IV-A,
// eqs. initbeta, initu, lanczos, with the LSQR updates), for P <= 64.
//
// A single workgroup keeps everything in LDS for the whole solve: the
// real-embedded steering vectors of the free pixels, the Ut fragments of u,
// and the vectors v, w, x; each lane keeps the u elements it owns in
// registers.  One step is, with only workgroup barriers:
//   F  u <- Psi_F v - (alpha/beta) u over the upper-triangle 16 x 16 tiles of
//      G = X_F diag(v) X_F^T (tiles spread over the four waves), fragments
//      of Ut written to LDS, ||u||^2;
//   A  g = x^T Ut x for every free pixel with the block-triangular form
//      x^T Ut x = sum_m x_m^T Ut_mm x_m + 2 sum_{k<m} x_m^T Ut_mk x_k, so only
//      the row tiles m >= k of each k tile are multiplied;
//      v_raw = g / beta - beta v, ||v_raw||^2;
//   S  FP64 rotation, vector updates and the stopping tests.
// The first pass sets u = b.  Tile indices are compile-time constants (the
// kernel is instantiated per row-tile count MT), so the register arrays of the
// row slices are never indexed dynamically.
#include "os_tiles.h"

namespace clsimg {

constexpr int kCuLds = 36864;  // floats of LDS (144 KiB)

__host__ __device__ constexpr int cu_row_stride(int Pp) { return 2 * Pp + ((18 - (2 * Pp) % 32) + 32) % 32; }

__host__ __device__ inline int cu_lds_floats(int MT, int n) {
  const int n16 = (n + 15) & ~15;
  return n16 * cu_row_stride(8 * MT) + 256 * MT * MT + 4 * n16;
}

// triangle tile t -> (mt, nt), mt <= nt, row by row (compile-time when t is)
__host__ __device__ constexpr int tri_row(int t, int MT) {
  int mt = 0;
  while (t >= MT - mt) {
    t -= MT - mt;
    ++mt;
  }
  return mt;
}
__host__ __device__ constexpr int tri_col(int t, int MT) {
  int mt = 0;
  while (t >= MT - mt) {
    t -= MT - mt;
    ++mt;
  }
  return mt + t;
}

template <int MT, int W>
__device__ inline void cu_forward(const float* xr, const float* vv, int n16, int RS, v4f* acc) {
  constexpr int NTP = MT * (MT + 1) / 2;
  constexpr int TPW = (NTP + 3) / 4;
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
#pragma unroll
  for (int i = 0; i < TPW; ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int kk = 0; kk < n16; kk += 4) {
    const int k = kk + q;
    const float vk = vv[k];
    float xm[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) xm[m] = xr[k * RS + 16 * m + c16];
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = W + 4 * i;
      if (t < NTP) {
        const int mt = tri_row(t, MT), nt = tri_col(t, MT);
        acc[i] = mfma16x16x4(xm[mt] * vk, xm[nt], acc[i]);
      }
    }
  }
}

// Ut fragment entry (row, col), kept only for col tile <= row tile, off-diagonal
// tiles doubled (block-triangular form of x^T Ut x)
__device__ inline void cu_put_frag(float* fr, int KS, int row, int col, float v) {
  const int rt = row >> 4, kt = col >> 4;
  if (kt > rt) return;
  fr[((rt * KS + (col >> 2)) * 64) + (col & 3) * 16 + (row & 15)] = (kt < rt) ? 2.f * v : v;
}

template <int MT, int W>
__device__ inline double cu_store_u(const v4f* acc, float2 (*uown)[4], float cu, bool first, int P,
                                    float* fr) {
  constexpr int NTP = MT * (MT + 1) / 2;
  constexpr int TPW = (NTP + 3) / 4;
  constexpr int KS = 4 * MT;
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
  double nrm = 0.0;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = W + 4 * i;
    if (t >= NTP) continue;
    const int mt = tri_row(t, MT), nt = tri_col(t, MT);
    const OsSlots sl = os_slots(mt, nt, c16, q, P, true);
    float2 K[4];
    os_assemble(first ? v4f{0.f, 0.f, 0.f, 0.f} : acc[i], sl, K);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (!sl.live[s]) continue;
      const int pa = sl.pa[s], pb = sl.pb[s];
      float2 r = make_float2(0.f, 0.f);
      if (pa < P && pb < P) {
        if (!first) {
          uown[i][s].x = K[s].x + cu * uown[i][s].x;
          uown[i][s].y = K[s].y + cu * uown[i][s].y;
        }
        r = uown[i][s];
        nrm += (double)r.x * r.x + (double)r.y * r.y;
      }
      cu_put_frag(fr, KS, 2 * pa, 2 * pb, r.x);
      cu_put_frag(fr, KS, 2 * pa, 2 * pb + 1, -r.y);
      cu_put_frag(fr, KS, 2 * pa + 1, 2 * pb, r.y);
      cu_put_frag(fr, KS, 2 * pa + 1, 2 * pb + 1, r.x);
    }
  }
  return nrm;
}

template <int MT, int W>
__device__ inline void cu_load_u(float2 (*uown)[4], const float2* B, int P) {
  constexpr int NTP = MT * (MT + 1) / 2;
  constexpr int TPW = (NTP + 3) / 4;
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = W + 4 * i;
    const bool act = t < NTP;
    const OsSlots sl = os_slots(act ? tri_row(t, MT) : 0, act ? tri_col(t, MT) : 0, c16, q, P, act);
    // Hermitian part of b, so that u and Ut stay exactly Hermitian / symmetric
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      uown[i][s] = make_float2(0.f, 0.f);
      if (sl.live[s] && sl.pa[s] < P && sl.pb[s] < P) {
        const float2 x = B[sl.pa[s] * P + sl.pb[s]], y = B[sl.pb[s] * P + sl.pa[s]];
        uown[i][s] = make_float2(0.5f * (x.x + y.x), 0.5f * (x.y - y.y));
      }
    }
  }
}

// g for the free pixels of 16-column tile j (all four row-halves in this wave)
template <int MT>
__device__ inline float cu_beam_tile(const float* xr, const float* fr, int RS, int col, bool valid) {
  constexpr int KS = 4 * MT;
  const int lane = threadIdx.x & 63, q = lane >> 4;
  v4f acc[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = v4f{0.f, 0.f, 0.f, 0.f};
  const float* xc = xr + col * RS;
#pragma unroll
  for (int kt = 0; kt < MT; ++kt) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kc = 4 * kt + j;
      const float b = valid ? xc[4 * kc + q] : 0.f;
#pragma unroll
      for (int m = kt; m < MT; ++m) acc[m] = mfma16x16x4(fr[(m * KS + kc) * 64 + lane], b, acc[m]);
    }
  }
  float gp = 0.f;
  if (valid) {
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const float* xm = xc + 16 * m + 4 * q;
      gp += xm[0] * acc[m][0] + xm[1] * acc[m][1] + xm[2] * acc[m][2] + xm[3] * acc[m][3];
    }
  }
  gp += __shfl_xor(gp, 16, 64);
  gp += __shfl_xor(gp, 32, 64);
  return gp;
}

template <int MT>
__global__ __launch_bounds__(kThreads) void lsqr_cu_kernel(LsqrCuParams pr) {
  constexpr int Pp = 8 * MT;
  constexpr int RS = cu_row_stride(Pp);
  constexpr int NTP = MT * (MT + 1) / 2;
  constexpr int TPW = (NTP + 3) / 4;
  __shared__ float lds[kCuLds];
  __shared__ double red[4];
  __shared__ double sc[8];
  __shared__ int s_done;
  __shared__ LsqrState sS;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c16 = lane & 15;
  const int P = pr.P, n = pr.n;
  const int n16 = (n + 15) & ~15;
  float* xr = lds;
  float* fr = xr + n16 * RS;
  float* vv = fr + 256 * MT * MT;
  float* ww = vv + n16;
  float* xv = ww + n16;
  float* vr = xv + n16;

  for (int e = tid; e < n16 * 2 * Pp; e += kThreads) {
    const int k = e / (2 * Pp), r = e - k * (2 * Pp);
    xr[k * RS + r] = k < n ? pr.xf[(size_t)k * 2 * Pp + r] : 0.f;
  }
  for (int e = tid; e < 4 * n16; e += kThreads) vv[e] = 0.f;
  for (int e = tid; e < 256 * MT * MT; e += kThreads) fr[e] = 0.f;
  float2 uown[TPW][4];
  switch (w) {
    case 0: cu_load_u<MT, 0>(uown, pr.B, P); break;
    case 1: cu_load_u<MT, 1>(uown, pr.B, P); break;
    case 2: cu_load_u<MT, 2>(uown, pr.B, P); break;
    default: cu_load_u<MT, 3>(uown, pr.B, P); break;
  }
  if (tid == 0) {
    LsqrState S = {};
    S.atol = pr.atol;
    S.btol = pr.btol;
    S.conlim = pr.conlim;
    S.itnlim = pr.itnlim;
    sS = S;
  }
  __syncthreads();
  float cu = 0.f;
  bool first = true;
  for (int it = 0;; ++it) {
    // ---- F: u <- Psi_F v - (alpha/beta) u (u = b on the first pass) ----
    double nb;
    {
      v4f acc[TPW];
      switch (w) {
        case 0:
          if (!first) cu_forward<MT, 0>(xr, vv, n16, RS, acc);
          nb = cu_store_u<MT, 0>(acc, uown, cu, first, P, fr);
          break;
        case 1:
          if (!first) cu_forward<MT, 1>(xr, vv, n16, RS, acc);
          nb = cu_store_u<MT, 1>(acc, uown, cu, first, P, fr);
          break;
        case 2:
          if (!first) cu_forward<MT, 2>(xr, vv, n16, RS, acc);
          nb = cu_store_u<MT, 2>(acc, uown, cu, first, P, fr);
          break;
        default:
          if (!first) cu_forward<MT, 3>(xr, vv, n16, RS, acc);
          nb = cu_store_u<MT, 3>(acc, uown, cu, first, P, fr);
          break;
      }
    }
    const double beta = sqrt(block_sum_d(nb, red));  // barrier inside: fragments complete
    // ---- A: v_raw = Psi_F^H u / beta - beta v ----
    double a2 = 0.0;
    for (int j = w; 16 * j < n; j += 4) {
      const int col = 16 * j + c16;
      const bool valid = col < n;
      const float g = cu_beam_tile<MT>(xr, fr, RS, col, valid);
      if (lane < 16 && valid) {
        double v = beta > 0.0 ? (double)g / beta : 0.0;
        if (!first) v -= beta * (double)vv[col];
        const float vf = (float)v;
        vr[col] = vf;
        a2 += (double)vf * vf;
      }
    }
    const double alpha = sqrt(block_sum_d(a2, red));
    // ---- S: rotation, vector updates and stopping tests ----
    if (tid == 0) {
      sc[0] = alpha > 0.0 ? 1.0 / alpha : 0.0;
      if (!first) {
        const double rho = hypot(sS.rhobar, beta);
        const double c = sS.rhobar / rho, sn = beta / rho;
        sc[1] = 1.0 / rho;         // d = w / rho
        sc[2] = c * sS.phibar;     // phi
        sc[3] = sn * alpha / rho;  // theta / rho
        sc[4] = c;
        sc[5] = sn;
      }
    }
    __syncthreads();
    const double iv = sc[0];
    double dd = 0.0, xx = 0.0;
    if (first) {
      for (int k = tid; k < n; k += kThreads) {
        const float vf = (float)((double)vr[k] * iv);
        vv[k] = vf;
        ww[k] = vf;
        xv[k] = 0.f;
      }
    } else {
      const double ir = sc[1], phi = sc[2], tr = sc[3];
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
        const double c = sc[4], sn = sc[5];
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
  for (int k = tid; k < n; k += kThreads) pr.x_out[k] = xv[k];
  __syncthreads();
  if (tid == 0) {
    *pr.Sfinal = sS;
    *pr.done = 1;
  }
}

bool lsqr_cu_fits(int P, int n) {
  const int MT = pad_p(P) / 8;
  return MT <= 8 && n > 0 && cu_lds_floats(MT, n) <= kCuLds;
}

hipError_t launch_lsqr_cu(const LsqrCuParams& pr, hipStream_t st) {
  const dim3 g(1), b(kThreads);
  switch (pad_p(pr.P) / 8) {
    case 1: hipLaunchKernelGGL(lsqr_cu_kernel<1>, g, b, 0, st, pr); break;
    case 2: hipLaunchKernelGGL(lsqr_cu_kernel<2>, g, b, 0, st, pr); break;
    case 3: hipLaunchKernelGGL(lsqr_cu_kernel<3>, g, b, 0, st, pr); break;
    case 4: hipLaunchKernelGGL(lsqr_cu_kernel<4>, g, b, 0, st, pr); break;
    case 5: hipLaunchKernelGGL(lsqr_cu_kernel<5>, g, b, 0, st, pr); break;
    case 6: hipLaunchKernelGGL(lsqr_cu_kernel<6>, g, b, 0, st, pr); break;
    case 7: hipLaunchKernelGGL(lsqr_cu_kernel<7>, g, b, 0, st, pr); break;
    case 8: hipLaunchKernelGGL(lsqr_cu_kernel<8>, g, b, 0, st, pr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace clsimg
