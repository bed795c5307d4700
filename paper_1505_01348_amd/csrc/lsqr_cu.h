// One LSQR solve of the free-set subproblem on one compute unit (Sec. IV-A,
// eqs. initbeta, initu, lanczos, with the LSQR updates), for P <= 48.
//
// A single workgroup keeps everything in LDS for the whole solve: the
// real-embedded steering vectors of the free pixels, the Ut fragments of u,
// and the vectors v, w, x; each lane keeps the u elements it owns in
// registers.  One step is, with only workgroup barriers:
//   F  u <- Psi_F v - (alpha/beta) u over the upper-triangle 16 x 16 tiles of
//      G = X_F diag(v) X_F^T (tiles spread over the 8 waves), fragments
//      of Ut written to LDS, ||u||^2;
//   A  g = x^T Ut x for every free pixel with the block-triangular form
//      x^T Ut x = sum_m x_m^T Ut_mm x_m + 2 sum_{k<m} x_m^T Ut_mk x_k, so only
//      the row tiles m >= k of each k tile are multiplied;
//      v_raw = g / beta - beta v, ||v_raw||^2;
//   S  FP64 rotation, vector updates and the stopping tests.
// Each phase ends in one block sum (one barrier), two per step.
// The first pass sets u = b.  Operands are read from LDS at run-time tile
// offsets; only the per-tile accumulators and owned u elements sit in
// register arrays, always at compile-time indices.  Shared by the LSQR-only
// kernel and the device-resident outer step.
#pragma once

#include "os_tiles.h"

namespace clsimg {

constexpr int kCuLds = 36864;  // floats of LDS (144 KiB)
constexpr int kCuThreads = 512;
constexpr int kCuWaves = kCuThreads / 64;

__host__ __device__ constexpr int cu_row_stride(int Pp) { return 2 * Pp + ((18 - (2 * Pp) % 32) + 32) % 32; }

__host__ __device__ inline int cu_lds_floats(int MT, int n) {
  const int n16 = (n + 15) & ~15;
  return n16 * cu_row_stride(8 * MT) + 256 * MT * MT + 4 * n16;
}

// G tile (mt, nt) = sum_k x_k[16mt + .] (vs v_k) x_k[16nt + .]^T over the n16 LDS
// rows: sixteen rows per step, all operands loaded before the four MFMAs
// (four accumulators)
__device__ inline v4f cu_forward_tile(const float* xr, const float* vv, float vs, int n16, int RS, int mt,
                                      int nt) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
  v4f acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
  const float* xa = xr + q * RS + 16 * mt + c16;
  const float* xb = xr + q * RS + 16 * nt + c16;
  for (int kk = 0; kk < n16; kk += 16) {
    float a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int o = (kk + 4 * u) * RS;
      a[u] = xa[o] * (vv[kk + 4 * u + q] * vs);
      b[u] = xb[o];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = mfma16x16x4(a[u], b[u], acc[u]);
  }
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}


// All NT triangle tiles of this wave in one pass over the rows (two
// accumulators each), so each step has 2 NT independent MFMAs.
template <int NT>
__device__ inline void cu_forward_tiles(const float* xr, const float* vv, float vs, int n16, int RS, const int* mt,
                                        const int* nt, v4f* out) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
  v4f acc[NT][2];
#pragma unroll
  for (int i = 0; i < NT; ++i) acc[i][0] = acc[i][1] = v4f{0.f, 0.f, 0.f, 0.f};
  const float* x0 = xr + q * RS + c16;
  for (int kk = 0; kk < n16; kk += 8) {
    const int o0 = kk * RS, o1 = (kk + 4) * RS;
    const float v0 = vv[kk + q] * vs, v1 = vv[kk + 4 + q] * vs;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      const float* xa = x0 + 16 * mt[i];
      const float* xb = x0 + 16 * nt[i];
      acc[i][0] = mfma16x16x4(xa[o0] * v0, xb[o0], acc[i][0]);
      acc[i][1] = mfma16x16x4(xa[o1] * v1, xb[o1], acc[i][1]);
    }
  }
#pragma unroll
  for (int i = 0; i < NT; ++i) out[i] = acc[i][0] + acc[i][1];
}

// Ut fragment entry (row, col), kept only for col tile <= row tile, off-diagonal
// tiles doubled (block-triangular form of x^T Ut x)
__device__ inline void cu_put_frag(float* fr, int KS, int row, int col, float v) {
  const int rt = row >> 4, kt = col >> 4;
  if (kt > rt) return;
  fr[((rt * KS + (col >> 2)) * 64) + (col & 3) * 16 + (row & 15)] = (kt < rt) ? 2.f * v : v;
}

// u <- K + cu * u on the owned elements (u kept when first), fragments of Ut;
// returns the owned part of ||u||^2
__device__ inline double cu_store_u(v4f acc, float2* uown, float cu, bool first, int P, int mt, int nt,
                                    int KS, float* fr) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
  const OsSlots sl = os_slots(mt, nt, c16, q, P, true);
  float2 K[4];
  os_assemble(acc, sl, K);
  double nrm = 0.0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (!sl.live[s]) continue;
    const int pa = sl.pa[s], pb = sl.pb[s];
    float2 r = make_float2(0.f, 0.f);
    if (pa < P && pb < P) {
      if (!first) {
        uown[s].x = K[s].x + cu * uown[s].x;
        uown[s].y = K[s].y + cu * uown[s].y;
      }
      r = uown[s];
      nrm += (double)r.x * r.x + (double)r.y * r.y;
    }
    cu_put_frag(fr, KS, 2 * pa, 2 * pb, r.x);
    cu_put_frag(fr, KS, 2 * pa, 2 * pb + 1, -r.y);
    cu_put_frag(fr, KS, 2 * pa + 1, 2 * pb, r.y);
    cu_put_frag(fr, KS, 2 * pa + 1, 2 * pb + 1, r.x);
  }
  return nrm;
}

// Hermitian part of the owned elements of b, so that u and Ut stay exactly
// Hermitian / symmetric
__device__ inline void cu_load_u(float2* uown, const float2* B, int P, int mt, int nt) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
  const OsSlots sl = os_slots(mt, nt, c16, q, P, true);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    uown[s] = make_float2(0.f, 0.f);
    if (sl.live[s] && sl.pa[s] < P && sl.pb[s] < P) {
      const float2 x = B[sl.pa[s] * P + sl.pb[s]], y = B[sl.pb[s] * P + sl.pa[s]];
      uown[s] = make_float2(0.5f * (x.x + y.x), 0.5f * (x.y - y.y));
    }
  }
}

// g for the 16 pixels of column tile col - c16 (all four row-quarters in this
// wave); rows beyond n are zero in LDS, so every load is unconditional.
template <int MT>
__device__ inline float cu_beam_tile(const float* xr, const float* fr, int RS, int col) {
  constexpr int KS = 4 * MT;
  const int lane = threadIdx.x & 63, q = lane >> 4;
  const float* xc = xr + col * RS;
  float b[KS];
#pragma unroll
  for (int kc = 0; kc < KS; ++kc) b[kc] = xc[4 * kc + q];
  v4f acc[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < MT; ++kt) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kc = 4 * kt + j;
#pragma unroll
      for (int m = kt; m < MT; ++m) acc[m] = mfma16x16x4(fr[(m * KS + kc) * 64 + lane], b[kc], acc[m]);
    }
  }
  float gp = 0.f;
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const float* xm = xc + 16 * m + 4 * q;
    gp += xm[0] * acc[m][0] + xm[1] * acc[m][1] + xm[2] * acc[m][2] + xm[3] * acc[m][3];
  }
  gp += __shfl_xor(gp, 16, 64);
  gp += __shfl_xor(gp, 32, 64);
  return gp;
}

// Block sum of NV doubles: DPP wave sums, one slot per wave in sh, one
// barrier.  Two reductions that alternate between two sh buffers never race:
// every reader of one buffer has passed the other buffer's barrier before
// that buffer is written again.
template <int NV>
__device__ inline void cu_block_sum(double (&v)[NV], double (*sh)[kCuWaves]) {
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum_dpp_d(v[i]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[i][w] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kCuWaves; ++k) t += sh[i][k];
    v[i] = t;
  }
}

// One pass of the F phase over this wave's triangle tiles (v = vs * vsrc);
// returns this thread's part of ||u||^2.
template <int TPW, int NTP>
__device__ inline double cu_phase_f(const float* xr, const float* vsrc, float vs, int n16, int RS, int P,
                                    int KS, const int* tmt, const int* tnt, float2 (*uown)[4], float cu,
                                    bool first, float* fr) {
  const int w = threadIdx.x >> 6;
  double nb = 0.0;
  v4f acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
  const int ntw = (NTP - w + kCuWaves - 1) / kCuWaves;  // tiles of this wave
  if (!first) {
    if (ntw == TPW) cu_forward_tiles<TPW>(xr, vsrc, vs, n16, RS, tmt, tnt, acc);
    else if (TPW > 1 && ntw == TPW - 1) cu_forward_tiles<(TPW > 1 ? TPW - 1 : 1)>(xr, vsrc, vs, n16, RS, tmt, tnt, acc);
  }
#pragma unroll
  for (int i = 0; i < TPW; ++i)
    if (w + kCuWaves * i < NTP) nb += cu_store_u(acc[i], uown[i], cu, first, P, tmt[i], tnt[i], KS, fr);
  return nb;
}

__host__ __device__ inline float* cu_x(float* lds, int MT, int n) {
  const int n16 = (n + 15) & ~15;
  return lds + n16 * cu_row_stride(8 * MT) + 256 * MT * MT + 2 * n16;
}

// The step order is the usual one; the only change is where the stopping
// tests of step k are evaluated: ||d_k||^2 and ||x_k||^2 are summed together
// with ||u_{k+1}||^2, so the F phase of step k+1 runs before the tests of step
// k and is discarded when they stop the iteration (x_k is untouched by it).
// Every thread keeps its own copy of the FP64 scalars; they are computed from
// the same block sums in the same order, so the copies agree bit for bit.
//
// cu_lsqr runs the whole solve inside the calling workgroup (kCuThreads
// threads).  On entry rows 0 .. n16 - 1 of the steering vectors must be in
// lds (stride cu_row_stride(8 MT), rows n .. n16 - 1 zero) and visible to all
// threads; on return the iterate x is at cu_x(lds, MT, n) and the returned
// state (identical in every thread) holds the scalars of the last step.
template <int MT>
__device__ LsqrState cu_lsqr(float* lds, int n, int P, const float2* __restrict__ B, double atol, double btol,
                             double conlim, int itnlim) {
  constexpr int Pp = 8 * MT;
  constexpr int KS = 4 * MT;
  constexpr int RS = cu_row_stride(Pp);
  constexpr int NTP = MT * (MT + 1) / 2;
  constexpr int TPW = (NTP + kCuWaves - 1) / kCuWaves;  // triangle tiles per wave (at most)
  __shared__ double redF[3][kCuWaves], redA[1][kCuWaves];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c16 = lane & 15;
  const int n16 = (n + 15) & ~15;
  float* xr = lds;
  float* fr = xr + n16 * RS;
  float* vv = fr + 256 * MT * MT;  // v
  float* ww = vv + n16;            // w
  float* xv = ww + n16;            // x
  float* vr = xv + n16;            // alpha * next v (zero beyond n)

  for (int e = tid; e < 4 * n16; e += kCuThreads) vv[e] = 0.f;
  for (int e = tid; e < 256 * MT * MT; e += kCuThreads) fr[e] = 0.f;
  // this wave's triangle tiles t = w + kCuWaves * i and the u elements it owns
  int tmt[TPW], tnt[TPW];
  float2 uown[TPW][4];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = w + kCuWaves * i;
    tri_tile(t < NTP ? t : 0, MT, tmt[i], tnt[i]);
    if (t < NTP) cu_load_u(uown[i], B, P, tmt[i], tnt[i]);
  }
  __syncthreads();

  // A phase: vr = Psi_F^H u / bet - bet v; returns ||vr||
  auto phase_a = [&](double bet) {
    double a2 = 0.0;
    for (int j = w; 16 * j < n; j += kCuWaves) {
      const int col = 16 * j + c16;
      const float g = cu_beam_tile<MT>(xr, fr, RS, col);
      if (lane < 16 && col < n) {
        const float vf = (float)((bet > 0.0 ? (double)g / bet : 0.0) - bet * (double)vv[col]);
        vr[col] = vf;
        a2 += (double)vf * vf;
      }
    }
    double r[1] = {a2};
    cu_block_sum<1>(r, redA);
    return (sqrt(r[0]));
  };

  double alpha, beta, rhobar, phibar, bnorm, rnorm, arnorm;
  double anorm2 = 0.0, ddnorm = 0.0, anorm = 0.0, acond = 0.0, xnorm = 0.0;
  int istop, itn = 0;

  // beta u = b, alpha v = Psi_F^H u
  {
    double r[3] = {cu_phase_f<TPW, NTP>(xr, vr, 0.f, n16, RS, P, KS, tmt, tnt, uown, 0.f, true, fr), 0.0,
                   0.0};
    cu_block_sum<3>(r, redF);
    beta = sqrt(r[0]);
  }
  alpha = phase_a(beta);
  rhobar = alpha;
  phibar = beta;
  bnorm = beta;
  rnorm = beta;
  arnorm = alpha * beta;
  istop = (alpha == 0.0 || beta == 0.0) ? 4 : 0;
  float ivf = alpha > 0.0 ? (float)(1.0 / alpha) : 0.f;
  for (int k = tid; k < n; k += kCuThreads) {
    const float vf = vr[k] * ivf;
    vv[k] = vf;
    ww[k] = vf;
    xv[k] = 0.f;
  }
  double dd = 0.0, xx = 0.0;  // this thread's part of ||d||^2 and ||x||^2 of the last step
  for (int it = 1; istop == 0; ++it) {
    // F: u <- Psi_F v - (alpha/beta) u, with v taken as vr * (1/alpha), the
    // same FP32 product the vector update stores in vv
    const float cu = beta > 0.0 ? (float)(-alpha / beta) : 0.f;
    double r[3] = {cu_phase_f<TPW, NTP>(xr, vr, ivf, n16, RS, P, KS, tmt, tnt, uown, cu, false, fr), dd, xx};
    cu_block_sum<3>(r, redF);
    if (it > 1) {  // stopping tests of step it - 1
      ddnorm = (ddnorm + r[1]);
      xnorm = sqrt(r[2]);
      anorm = sqrt(anorm2);
      acond = (anorm * sqrt(ddnorm));
      if (rnorm <= btol * bnorm + atol * anorm * xnorm) istop = 1;
      else if (arnorm <= atol * anorm * rnorm) istop = 2;
      else if (acond >= conlim) istop = 3;
      else if (alpha == 0.0 || beta == 0.0) istop = 4;
      else if (itn >= itnlim) istop = 7;
      if (istop) break;
    }
    const double beta_n = sqrt(r[0]);
    const double alpha_n = phase_a(beta_n);
    // plane rotation and the updates of w and x
    anorm2 += alpha * alpha + beta_n * beta_n;
    const double rho = hypot(rhobar, beta_n);
    const double c = (rhobar / rho), sn = (beta_n / rho);
    const double phi = (c * phibar);
    const double ir = (1.0 / rho), tr = (sn * alpha_n / rho);
    rhobar = (-c * alpha_n);
    phibar = (sn * phibar);
    alpha = alpha_n;
    beta = beta_n;
    rnorm = phibar;
    arnorm = (phibar * alpha * fabs(c));
    itn = it;
    ivf = alpha > 0.0 ? (float)(1.0 / alpha) : 0.f;
    dd = 0.0;
    xx = 0.0;
    for (int k = tid; k < n; k += kCuThreads) {
      const float vf = vr[k] * ivf;
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
  LsqrState S = {};
  S.alpha = alpha;
  S.beta = beta;
  S.rhobar = rhobar;
  S.phibar = phibar;
  S.bnorm = bnorm;
  S.anorm2 = anorm2;
  S.ddnorm = ddnorm;
  S.rnorm = rnorm;
  S.arnorm = arnorm;
  S.anorm = anorm;
  S.acond = acond;
  S.xnorm = xnorm;
  S.atol = atol;
  S.btol = btol;
  S.conlim = conlim;
  S.itn = itn;
  S.itnlim = itnlim;
  S.istop = istop;
  S.done = 1;
  return S;
}

}  // namespace clsimg
