// Device-resident outer iteration of the active-set method (Table I) for
// P <= 48 and free sets that fit in one workgroup's LDS.
//
// Every outer step changes the free set by one pixel (an add after a feasible
// step, a block after an infeasible one), so one workgroup can carry the whole
// step: it keeps the sorted lists of F and U, applies the decision taken from
// the Lagrange multipliers of the previous feasible step, forms
// b = B0 - Psi_U gamma_U (eq. bsubproblemLS) when U changed, generates the
// steering vectors of F from the separable tables, runs LSQR (Sec. IV-A), and
// takes the feasible step (sigma_F = z, then E = Psi_F sigma_F - b for the
// gradient, eq. gls) or the infeasible one (eq. mumax).  The multipliers of a
// feasible step (eqs. etaL, etaU) come from the full-grid beamformer, which
// runs between two outer steps and leaves one partial argmin key per block.
//
// The host enqueues (outer step, multipliers) pairs in batches and reads the
// state once per batch; steps enqueued after the iteration stopped return at
// once.  When a free set outgrows the LDS, the outer step stops with
// `fallback` set and the host continues with its own loop from the current
// sigma and state.
//
// PWLS (eq. preWLS) runs the same step on the transformed problem: steering
// rows L^-1 a_i / sqrt(D_i) (R = L L^H, D_i = h_i^2 / C), data L^-1 B0 L^-H,
// bound D gamma; the gradient matrix E of the whitened problem is handed to
// the multiplier kernel as L^-H E L^-1 with a per-pixel factor 1 / D_i.
#include <algorithm>

#include "../../include/clsimg.h"
#include "lsqr_cu.h"

namespace clsimg {

constexpr int kOuterMaxF = 1024;  // entries of the LDS copy of the free list
constexpr int kPerThread = kOuterMaxF / kCuThreads;  // list entries each thread moves in a shift
static_assert(kOuterMaxF % kCuThreads == 0, "list shifts assume whole entries per thread");

__device__ inline int cu_block_sum_i(int v, int (&sh)[kCuWaves]) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  int s = 0;
#pragma unroll
  for (int i = 0; i < kCuWaves; ++i) s += sh[i];
  return s;
}

__device__ inline int cu_block_min_i(int v, int (&sh)[kCuWaves]) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  int s = sh[0];
#pragma unroll
  for (int i = 1; i < kCuWaves; ++i) s = min(s, sh[i]);
  return s;
}

__device__ inline float cu_block_min_f(float v, float (&sh)[kCuWaves]) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = sh[0];
#pragma unroll
  for (int i = 1; i < kCuWaves; ++i) s = fminf(s, sh[i]);
  return s;
}

// order-preserving map of a double to uint64 (no NaN arrives here)
__device__ inline uint64_t ordered_bits_d(double d) {
  const uint64_t u = (uint64_t)__double_as_longlong(d);
  return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__device__ inline double from_ordered_bits_d(uint64_t u) {
  const uint64_t v = (u & 0x8000000000000000ull) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u;
  return __longlong_as_double((long long)v);
}

// Real-embedded steering vectors of pixels list[0 .. n) into LDS rows
// (x[2p] = Re a_p, x[2p+1] = Im a_p, rows n .. n16 - 1 zero), optionally with
// the row weights w[k] = wsrc[list[k]].
template <int MT>
__device__ inline void cu_gen_rows(const Tables& tab, const int* list, int n, float* xr, const float* wsrc,
                                   float* w) {
  constexpr int Pp = 8 * MT;
  constexpr int RS = cu_row_stride(Pp);
  const int n16 = (n + 15) & ~15;
  for (int e = threadIdx.x; e < n16 * Pp; e += kCuThreads) {
    const int k = e / Pp, p = e - k * Pp;
    float2 a = make_float2(0.f, 0.f);
    if (k < n) {
      const int i = list[k];
      const int im = i / tab.nl, il = i - im * tab.nl;
      a = tab.a(p, il, im);
    }
    xr[k * RS + 2 * p] = a.x;
    xr[k * RS + 2 * p + 1] = a.y;
  }
  if (w)
    for (int k = threadIdx.x; k < n16; k += kCuThreads) w[k] = k < n ? wsrc[list[k]] : 0.f;
}

// PWLS rows: x_k <- rowscale[list[k]] * L^-1 x_k for the n LDS rows, in
// chunks of kWhChunk rows through the LDS scratch tmp (kWhChunk * 2Pp floats);
// Lw (LDS) holds L^-1 row-major as complex pairs.  Entries of padding antennas
// stay zero.
constexpr int kWhChunk = 16;
template <int MT>
__device__ inline void cu_whiten_rows(float* xr, const int* list, int n, const float2* Lw, float* tmp,
                                      const float* rowscale, int P) {
  constexpr int Pp = 8 * MT;
  constexpr int RS = cu_row_stride(Pp);
  for (int k0 = 0; k0 < n; k0 += kWhChunk) {
    const int nc = min(kWhChunk, n - k0);
    for (int e = threadIdx.x; e < nc * P; e += kCuThreads) {
      const int kk = e / P, p = e - kk * P;
      const float* row = xr + (k0 + kk) * RS;
      float re = 0.f, im = 0.f;
      for (int r = 0; r <= p; ++r) {  // L^-1 is lower triangular
        const float2 l = Lw[p * P + r];
        const float ar = row[2 * r], ai = row[2 * r + 1];
        re += l.x * ar - l.y * ai;
        im += l.x * ai + l.y * ar;
      }
      const float sc = rowscale[list[k0 + kk]];
      tmp[kk * 2 * Pp + 2 * p] = sc * re;
      tmp[kk * 2 * Pp + 2 * p + 1] = sc * im;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nc * 2 * P; e += kCuThreads) {
      const int kk = e / (2 * P), c = e - kk * 2 * P;
      xr[(k0 + kk) * RS + c] = tmp[kk * 2 * Pp + c];
    }
    __syncthreads();
  }
}

// L^-1 into LDS (P x P complex, row-major)
__device__ inline void cu_load_lw(const float2* __restrict__ Lw, int P, float2* dst) {
  for (int e = threadIdx.x; e < P * P; e += kCuThreads) dst[e] = Lw[e];
}

// out = sK K + sB herm(B) over this wave's owned elements, K from a forward
// tile; returns the sum of |out|^2 over them
__device__ inline double cu_store_c(v4f acc, int mt, int nt, int P, float sK, float sB,
                                    const float2* __restrict__ B, float2* out) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
  const OsSlots sl = os_slots(mt, nt, c16, q, P, true);
  float2 K[4];
  os_assemble(acc, sl, K);
  double nrm = 0.0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (!sl.live[s] || sl.pa[s] >= P || sl.pb[s] >= P) continue;
    const float2 x = B[sl.pa[s] * P + sl.pb[s]], y = B[sl.pb[s] * P + sl.pa[s]];
    const float2 o =
        make_float2(sK * K[s].x + sB * (0.5f * (x.x + y.x)), sK * K[s].y + sB * (0.5f * (x.y - y.y)));
    out[sl.pa[s] * P + sl.pb[s]] = o;
    nrm += (double)o.x * o.x + (double)o.y * o.y;
  }
  return nrm;
}

__device__ inline const int* ulist_cur(const OuterParams& pr, const OuterState& S) {
  return pr.Ulist + (size_t)S.ucur * pr.Q;
}

template <int MT>
__device__ void outer_step_body(const OuterParams& pr) {
  constexpr int Pp = 8 * MT;
  constexpr int RS = cu_row_stride(Pp);
  constexpr int NTP = MT * (MT + 1) / 2;
  constexpr int TPW = (NTP + kCuWaves - 1) / kCuWaves;
  __shared__ float lds[kCuLds];
  __shared__ int sF[kOuterMaxF];
  __shared__ OuterState S;
  __shared__ int shi[kCuWaves];
  __shared__ float shf[kCuWaves];
  __shared__ uint64_t shk[kCuWaves];
  __shared__ double shd[1][kCuWaves];
  __shared__ int s_add, s_from_u;
  const int tid = threadIdx.x, w = tid >> 6;
  const int P = pr.P, Q = pr.Q;
  if (tid == 0) S = *pr.st;
  __syncthreads();
  if (S.done) return;
  for (int k = tid; k < S.nF && k < kOuterMaxF; k += kCuThreads) sF[k] = pr.Flist[k];

  // ---- decision from the multipliers of the last feasible step ----
  if (S.await_lambda) {
    uint64_t m = ~0ull;
    for (int i = tid; i < pr.nkeys; i += kCuThreads) m = pr.keys[i] < m ? pr.keys[i] : m;
    m = block_min_u64(m, shk);
    if (tid == 0) {
      s_add = -1;
      s_from_u = 0;
      S.await_lambda = 0;
      if (m == ~0ull) {
        S.done = 1;  // no active pixel left
      } else {
        const float lam = from_ordered_bits((uint32_t)(m >> 32));
        const int i = (int)(m & 0xFFFFFFFFull);
        const float thr = pr.eps[i];
        S.last_imin = i;
        S.last_lam = lam;
        S.last_eps = thr;
        if (thr > 0.f) S.margin_lambda = fmin(S.margin_lambda, fabs((double)lam + thr) / thr);
        if (lam < -thr) {
          s_add = i;
          s_from_u = pr.state[i] == kStateU;
          pr.state[i] = kStateF;
          ++S.adds;
          S.last_added = i;
        } else {
          S.done = 1;
        }
      }
    }
    __syncthreads();
    const int add = s_add;
    if (add >= 0) {
      // insert into the sorted free list (LDS) ...
      const int n = S.nF;
      int cnt = 0;
      for (int k = tid; k < n && k < kOuterMaxF; k += kCuThreads) cnt += sF[k] < add;
      const int pos = cu_block_sum_i(cnt, shi);
      if (n < kOuterMaxF) {
        int v[kPerThread];
#pragma unroll
        for (int j = 0; j < kPerThread; ++j) {
          const int k = tid + j * kCuThreads;
          v[j] = k < n ? sF[k] : 0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kPerThread; ++j) {
          const int k = tid + j * kCuThreads;
          if (k < n && k >= pos) sF[k + 1] = v[j];
        }
        if (tid == 0) sF[pos] = add;
      }
      // ... and take it out of the upper-bound list (global, two buffers)
      if (s_from_u) {
        const int* Uo = ulist_cur(pr, S);
        int* Un = pr.Ulist + (size_t)(1 - S.ucur) * Q;
        int kp = 0x7fffffff;
        for (int k = tid; k < S.nU; k += kCuThreads)
          if (Uo[k] == add) kp = k;
        kp = cu_block_min_i(kp, shi);
        for (int k = tid; k < S.nU - 1; k += kCuThreads) Un[k] = k < kp ? Uo[k] : Uo[k + 1];
      }
      __syncthreads();
      if (tid == 0) {
        ++S.nF;
        if (s_from_u) {
          --S.nU;
          S.ucur = 1 - S.ucur;
          S.bb_dirty = 1;
        }
      }
    }
    __syncthreads();
  }

  // ||B0||^2 once (for the relative residual reported at the end)
  if (S.outer == 0 && !S.done) {
    double b2 = 0.0;
    for (int e = tid; e < P * P; e += kCuThreads) {
      const float2 v = pr.B0[e];
      b2 += (double)v.x * v.x + (double)v.y * v.y;
    }
    double r[1] = {b2};
    cu_block_sum<1>(r, shd);
    if (tid == 0) S.b0n2 = r[0];
    __syncthreads();
  }

  // ---- guards ----
  if (tid == 0 && !S.done) {
    if (S.outer >= pr.max_outer) {
      S.status = kStatusMaxOuter;
      S.done = 1;
    } else if (S.nF > kOuterMaxF || S.nF > pr.max_f ||
               cu_lds_floats(MT, S.nF) + (pr.Lw ? kWhChunk * 2 * Pp : 0) > kCuLds) {
      S.fallback = 1;
      S.done = 1;
    }
  }
  __syncthreads();
  const int n = S.nF, n16 = (n + 15) & ~15;
  auto finish = [&]() {
    __syncthreads();
    for (int k = tid; k < S.nF && k < kOuterMaxF; k += kCuThreads) pr.Flist[k] = sF[k];
    if (tid == 0) {
      S.lam_skip = !(S.await_lambda && !S.done);
      *pr.st = S;
    }
  };
  if (S.done) {
    finish();
    return;
  }

  // this wave's triangle tiles
  int tmt[TPW], tnt[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = w + kCuWaves * i;
    tri_tile(t < NTP ? t : 0, MT, tmt[i], tnt[i]);
  }

  // ---- b = B0 - Psi_U gamma_U, recomputed when U changed ----
  if (S.bb_dirty) {
    if (S.nU > 0) {
      const int* U = ulist_cur(pr, S);
      // rows per chunk, leaving room for L^-1 and the whitening scratch
      constexpr int CH = ((kCuLds - 64 - 2 * Pp * Pp - kWhChunk * 2 * Pp) / (RS + 1)) & ~15;
      float* xr = lds;
      float* wg = lds + CH * RS;
      float2* lw = reinterpret_cast<float2*>(wg + CH);
      float* wtmp = reinterpret_cast<float*>(lw + Pp * Pp);
      if (pr.Lw) cu_load_lw(pr.Lw, P, lw);
      v4f acc[TPW];
#pragma unroll
      for (int i = 0; i < TPW; ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
      for (int c0 = 0; c0 < S.nU; c0 += CH) {
        const int nc = min(CH, S.nU - c0), nc16 = (nc + 15) & ~15;
        cu_gen_rows<MT>(pr.tab, U + c0, nc, xr, pr.gamma, wg);
        __syncthreads();
        if (pr.Lw) cu_whiten_rows<MT>(xr, U + c0, nc, lw, wtmp, pr.rowscale, P);
#pragma unroll
        for (int i = 0; i < TPW; ++i)
          if (w + kCuWaves * i < NTP) acc[i] = acc[i] + cu_forward_tile(xr, wg, 1.f, nc16, RS, tmt[i], tnt[i]);
        __syncthreads();
      }
#pragma unroll
      for (int i = 0; i < TPW; ++i)
        if (w + kCuWaves * i < NTP) cu_store_c(acc[i], tmt[i], tnt[i], P, -1.f, 1.f, pr.B0, pr.Bb);
    }
    __syncthreads();
    if (tid == 0) {
      S.psi_flops += 8.0 * P * P * S.nU;
      S.bb_dirty = 0;
    }
  }
  const float2* bsub = S.nU > 0 ? pr.Bb : pr.B0;

  // ---- LSQR on the free set ----
  cu_gen_rows<MT>(pr.tab, sF, n, lds, nullptr, nullptr);
  if (pr.Lw) {  // PWLS: L^-1 in the (not yet used) fragment area, scratch after the vectors
    float2* lw = reinterpret_cast<float2*>(lds + n16 * RS);
    cu_load_lw(pr.Lw, P, lw);
    __syncthreads();
    cu_whiten_rows<MT>(lds, sF, n, lw, lds + cu_lds_floats(MT, n), pr.rowscale, P);
  }
  __syncthreads();
  const int itnlim = pr.itnlim < 0 ? 4 * n + 100 : pr.itnlim;
  const LsqrState L = cu_lsqr<MT>(lds, n, P, bsub, pr.atol, pr.btol, pr.conlim, itnlim);
  float* z = cu_x(lds, MT, n);
  __syncthreads();

  // ---- step (Table I) ----
  int ok = 1;
  float mz = 3.0e38f;
  for (int k = tid; k < n; k += kCuThreads) {
    const float zk = z[k], g = pr.gamma[sF[k]];
    ok &= (zk >= 0.f) && (zk <= g);
    mz = fminf(mz, fminf(zk, g - zk) / g);
  }
  ok = cu_block_min_i(ok, shi);
  mz = cu_block_min_f(mz, shf);
  if (ok) {
    // feasible: sigma_F = z, then E = Psi_F sigma_F - b on the owned elements;
    // ||E|| is the residual of this image
    for (int k = tid; k < n; k += kCuThreads) pr.sigma[sF[k]] = z[k];
    double e2 = 0.0;
#pragma unroll
    for (int i = 0; i < TPW; ++i)
      if (w + kCuWaves * i < NTP) {
        const v4f acc = cu_forward_tile(lds, z, 1.f, n16, RS, tmt[i], tnt[i]);
        e2 += cu_store_c(acc, tmt[i], tnt[i], P, 1.f, -1.f, bsub, pr.E);
      }
    {
      double r[1] = {e2};
      cu_block_sum<1>(r, shd);  // (its barrier also completes E)
      if (tid == 0) S.res2 = r[0];
    }
    __syncthreads();
    if (pr.Lw) {
      // PWLS: the multiplier kernel beamforms L^-H E L^-1 (and scales by 1/D)
      float2* Ed = reinterpret_cast<float2*>(lds);
      float2* lw = Ed + P * P;
      float2* T = lw + P * P;
      for (int e = tid; e < P * P; e += kCuThreads) {
        Ed[e] = pr.E[e];
        lw[e] = pr.Lw[e];
      }
      __syncthreads();
      for (int e = tid; e < P * P; e += kCuThreads) {  // T = E L^-1
        const int p = e / P, q = e - p * P;
        float re = 0.f, im = 0.f;
        for (int r = q; r < P; ++r) {
          const float2 a = Ed[p * P + r], l = lw[r * P + q];
          re += a.x * l.x - a.y * l.y;
          im += a.x * l.y + a.y * l.x;
        }
        T[e] = make_float2(re, im);
      }
      __syncthreads();
      for (int e = tid; e < P * P; e += kCuThreads) {  // E' = L^-H T
        const int p = e / P, q = e - p * P;
        float re = 0.f, im = 0.f;
        for (int r = p; r < P; ++r) {
          const float2 l = lw[r * P + p], t = T[r * P + q];  // conj(l) * t
          re += l.x * t.x + l.y * t.y;
          im += l.x * t.y - l.y * t.x;
        }
        pr.E[e] = make_float2(re, im);
      }
      __syncthreads();
    }
    if (tid == 0) {
      if (n > 0) S.margin_z = fmin(S.margin_z, (double)mz);
      S.last_feasible = 1;
      S.last_ib = -1;
      if (n >= Q) S.done = 1;  // no active pixel
      else S.await_lambda = 1;
      S.psi_flops += 8.0 * P * P * n + 8.0 * P * P * Q + 8.0 * P * Q;
    }
  } else {
    // infeasible: largest step along p = z - sigma_F, ties to the lowest pixel
    double best = INFINITY;
    for (int k = tid; k < n; k += kCuThreads) {
      const int i = sF[k];
      const double sg = pr.sigma[i], p = (double)z[k] - sg;
      if (p != 0.0) best = fmin(best, fmax(-sg / p, ((double)pr.gamma[i] - sg) / p));
    }
    const uint64_t kb = block_min_u64(ordered_bits_d(best), shk);
    best = from_ordered_bits_d(kb);
    int bk = 0x7fffffff;
    for (int k = tid; k < n; k += kCuThreads) {
      const int i = sF[k];
      const double sg = pr.sigma[i], p = (double)z[k] - sg;
      if (p != 0.0 && fmax(-sg / p, ((double)pr.gamma[i] - sg) / p) == best) bk = min(bk, k);
    }
    bk = cu_block_min_i(bk, shi);
    if (bk >= n) {  // no finite step (non-finite z): stop moving, block the first pixel
      bk = 0;
      best = 0.0;
    }
    const int ib = sF[bk];
    const double pb = (double)z[bk] - (double)pr.sigma[ib];  // read before sigma changes
    __syncthreads();
    for (int k = tid; k < n; k += kCuThreads) {
      const int i = sF[k];
      const double sg = pr.sigma[i], p = (double)z[k] - sg;
      pr.sigma[i] = (float)fmin(fmax(sg + best * p, 0.0), (double)pr.gamma[i]);
    }
    __syncthreads();
    const bool to_upper = !(pb < 0.0);
    if (tid == 0) {
      pr.sigma[ib] = to_upper ? pr.gamma[ib] : 0.f;
      pr.state[ib] = to_upper ? (uint8_t)kStateU : (uint8_t)kStateL;
      ++S.drops;
      S.last_feasible = 0;
      S.last_ib = ib;
      S.last_ib_to = to_upper ? kStateU : kStateL;
      S.last_mu = (float)best;
      if (ib == S.last_added && (float)best == 0.0f) {
        S.status = kStatusCycle;
        S.done = 1;
      }
    }
    // take ib out of the free list
    {
      int v[kPerThread];
#pragma unroll
      for (int j = 0; j < kPerThread; ++j) {
        const int k = tid + j * kCuThreads;
        v[j] = (k < n && k > bk) ? sF[k] : 0;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kPerThread; ++j) {
        const int k = tid + j * kCuThreads;
        if (k < n && k > bk) sF[k - 1] = v[j];
      }
    }
    // and into the upper-bound list
    if (to_upper) {
      const int* Uo = ulist_cur(pr, S);
      int* Un = pr.Ulist + (size_t)(1 - S.ucur) * Q;
      int cnt = 0;
      for (int k = tid; k < S.nU; k += kCuThreads) cnt += Uo[k] < ib;
      const int pos = cu_block_sum_i(cnt, shi);
      for (int k = tid; k <= S.nU; k += kCuThreads) Un[k] = k < pos ? Uo[k] : (k == pos ? ib : Uo[k - 1]);
    }
    __syncthreads();
    if (tid == 0) {
      --S.nF;
      if (to_upper) {
        ++S.nU;
        S.ucur = 1 - S.ucur;
        S.bb_dirty = 1;
      }
    }
  }
  if (tid == 0) {
    S.last_added = -1;
    ++S.outer;
    S.lsqr_total += L.itn;
    S.last_itn = L.itn;
    S.last_istop = L.istop;
    if (L.istop == 7) ++S.itnlim_hits;
    if (n > 0) S.psi_flops += (8.0 * P * P * n + 8.0 * P * n) + L.itn * (16.0 * P * P * n + 8.0 * P * n);
  }
  finish();
}

template <int MT>
__global__ __launch_bounds__(kCuThreads) void outer_step_kernel(OuterParams pr) {
  outer_step_body<MT>(pr);
}

// one workgroup per request of a batch (all with the same P)
template <int MT>
__global__ __launch_bounds__(kCuThreads) void outer_step_batch_kernel(const OuterParams* __restrict__ prs) {
  const OuterParams pr = prs[blockIdx.x];
  outer_step_body<MT>(pr);
}

__device__ OuterState fresh_outer_state(const SolveDecision* dec) {
  OuterState S = {};
  S.nF = dec ? dec->nF : 0;
  S.nU = dec ? dec->nU : 0;
  S.last_added = -1;
  S.bb_dirty = S.nU > 0;
  S.margin_lambda = INFINITY;
  S.margin_z = INFINITY;
  S.lam_skip = 1;
  S.last_ib = -1;
  S.last_imin = -1;
  return S;
}

__global__ void outer_init_kernel(OuterState* st, const SolveDecision* dec) {
  if (threadIdx.x != 0) return;
  *st = fresh_outer_state(dec);
}

// per blocks of 256 threads per request
__global__ __launch_bounds__(256) void request_init_batch_kernel(const ReqInitItem* __restrict__ items, int per) {
  const int r = blockIdx.x / per, b = blockIdx.x - r * per;
  const ReqInitItem it = items[r];
  const int t = b * 256 + threadIdx.x, nt = per * 256;
  for (int e = t; e < it.Q; e += nt) {
    it.sigma[e] = 0.f;
    it.state[e] = 0;
  }
  for (int e = t; e < it.P * it.P; e += nt) {
    float2 v = it.R[e];
    const int p = e / it.P, q = e - p * it.P;
    if (it.noise && p == q) v.x -= it.noise[p];
    it.B0[e] = v;
  }
  if (t == 0) *it.st = fresh_outer_state(nullptr);
}

// ---- PWLS set-up (eq. preWLS, eq. D at K = 1) ----
// D_i = h_i^2 / C; rowscale = 1 / sqrt(D); bound D gamma; threshold
// kd_coef / h_i (kd_coef = kappa_d / sqrt(N - P - 1), App. A); dinv = 1 / D.
__global__ void pwls_setup_kernel(const float* __restrict__ h, const float* __restrict__ gamma, double C,
                                  double kd_coef, int Q, float* __restrict__ rowscale, float* __restrict__ gamma_pw,
                                  float* __restrict__ eps_pw, float* __restrict__ dinv) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < Q; i += gridDim.x * blockDim.x) {
    const double hh = (double)h[i];
    const double D = hh * hh / C;
    rowscale[i] = (float)(sqrt(C) / hh);
    gamma_pw[i] = (float)(D * (double)gamma[i]);
    eps_pw[i] = (float)(kd_coef / hh);
    dinv[i] = (float)(1.0 / D);
  }
}

// L^-1 to FP32, and the whitened data L^-1 herm(B0) L^-H in FP64 (one workgroup)
__global__ __launch_bounds__(1024) void pwls_whiten_kernel(const double2* __restrict__ Li,
                                                           const float2* __restrict__ B0, int P,
                                                           float2* __restrict__ Lw, float2* __restrict__ B0w) {
  __shared__ double2 T[48 * 48];
  for (int e = threadIdx.x; e < P * P; e += blockDim.x) Lw[e] = make_float2((float)Li[e].x, (float)Li[e].y);
  for (int e = threadIdx.x; e < P * P; e += blockDim.x) {  // T = L^-1 herm(B0)
    const int p = e / P, q = e - p * P;
    double re = 0.0, im = 0.0;
    for (int r = 0; r <= p; ++r) {
      const double2 l = Li[p * P + r];
      const float2 x = B0[r * P + q], y = B0[q * P + r];
      const double br = 0.5 * ((double)x.x + y.x), bi = 0.5 * ((double)x.y - y.y);
      re += l.x * br - l.y * bi;
      im += l.x * bi + l.y * br;
    }
    T[e] = make_double2(re, im);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < P * P; e += blockDim.x) {  // B0w = T L^-H
    const int p = e / P, q = e - p * P;
    double re = 0.0, im = 0.0;
    for (int r = 0; r <= q; ++r) {
      const double2 t = T[p * P + r], l = Li[q * P + r];  // t * conj(l)
      re += t.x * l.x + t.y * l.y;
      im += t.y * l.x - t.x * l.y;
    }
    B0w[e] = make_float2((float)re, (float)im);
  }
}

// ---- PWLS on the host-driven loop (any P up to the Cholesky limit) ----
// out = M herm(X) M^H with M = L^-1 (whiten) or M = L^-H (colour), in two
// passes through an FP64 P x P temporary T: pass 1 T = M herm(X) (one
// workgroup per row of T), pass 2 out = T M^H (one workgroup per row of out,
// optionally that row's squared Frobenius norm in FP64).  L^-1 (Li, FP64,
// lower triangular, row-major) supplies both factors: for the whitening
// M[p][r] = Li[p][r] (r <= p) and M^H[r][q] = conj(Li[q][r]) (r <= q); for the
// colouring M[p][r] = conj(Li[r][p]) (r >= p) and M^H[r][q] = Li[r][q] (r >= q).
__global__ __launch_bounds__(256) void pwls_sandwich_left_kernel(const double2* __restrict__ Li,
                                                                 const float2* __restrict__ X, int P, int colour,
                                                                 double2* __restrict__ T) {
  const int p = blockIdx.x;
  for (int q = threadIdx.x; q < P; q += blockDim.x) {
    double re = 0.0, im = 0.0;
    const int r0 = colour ? p : 0, r1 = colour ? P - 1 : p;
    for (int r = r0; r <= r1; ++r) {
      double2 m = colour ? Li[(size_t)r * P + p] : Li[(size_t)p * P + r];
      if (colour) m.y = -m.y;
      const float2 x = X[(size_t)r * P + q], y = X[(size_t)q * P + r];  // herm(X)[r][q]
      const double br = 0.5 * ((double)x.x + y.x), bi = 0.5 * ((double)x.y - y.y);
      re += m.x * br - m.y * bi;
      im += m.x * bi + m.y * br;
    }
    T[(size_t)p * P + q] = make_double2(re, im);
  }
}

__global__ __launch_bounds__(256) void pwls_sandwich_right_kernel(const double2* __restrict__ Li,
                                                                  const double2* __restrict__ T, int P, int colour,
                                                                  float2* __restrict__ out, double* __restrict__ norm2) {
  __shared__ double part[256];
  const int p = blockIdx.x;
  double nn = 0.0;
  for (int q = threadIdx.x; q < P; q += blockDim.x) {
    double re = 0.0, im = 0.0;
    const int r0 = colour ? q : 0, r1 = colour ? P - 1 : q;
    for (int r = r0; r <= r1; ++r) {
      double2 m = colour ? Li[(size_t)r * P + q] : Li[(size_t)q * P + r];
      if (!colour) m.y = -m.y;
      const double2 t = T[(size_t)p * P + r];
      re += t.x * m.x - t.y * m.y;
      im += t.x * m.y + t.y * m.x;
    }
    const float2 o = make_float2((float)re, (float)im);
    out[(size_t)p * P + q] = o;
    nn += (double)o.x * o.x + (double)o.y * o.y;
  }
  if (!norm2) return;
  part[threadIdx.x] = nn;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) norm2[p] = part[0];
}

// The free set's steering rows whitened in place: x_k <- rowscale[F[k]] L^-1 x_k
// (xf layout: 2 Pp floats per pixel, padding antennas zero); one workgroup
// per row.
__global__ __launch_bounds__(128) void pwls_xf_whiten_kernel(const double2* __restrict__ Li, int P, int Pp,
                                                             const int* __restrict__ Flist, int n,
                                                             const float* __restrict__ rowscale,
                                                             float* __restrict__ xf) {
  __shared__ float2 x[CLSIMG_MAX_P];
  const int k = blockIdx.x;
  float2* row = reinterpret_cast<float2*>(xf + (size_t)k * 2 * Pp);
  for (int r = threadIdx.x; r < P; r += blockDim.x) x[r] = row[r];
  __syncthreads();
  const double sc = (double)rowscale[Flist[k]];
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int r = 0; r <= p; ++r) {
      const double2 l = Li[(size_t)p * P + r];
      const float2 v = x[r];
      re += l.x * v.x - l.y * v.y;
      im += l.x * v.y + l.y * v.x;
    }
    row[p] = make_float2((float)(sc * re), (float)(sc * im));
  }
}

hipError_t launch_pwls_sandwich(const double2* Li, const float2* X, int P, bool colour, double2* T, float2* out,
                                double* norm2, hipStream_t st) {
  if (P < 1 || P > CLSIMG_MAX_P) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pwls_sandwich_left_kernel, dim3(P), dim3(128), 0, st, Li, X, P, colour ? 1 : 0, T);
  hipLaunchKernelGGL(pwls_sandwich_right_kernel, dim3(P), dim3(128), 0, st, Li, (const double2*)T, P,
                     colour ? 1 : 0, out, norm2);
  return hipGetLastError();
}

hipError_t launch_pwls_xf_whiten(const double2* Li, int P, const int* Flist, int n, const float* rowscale, float* xf,
                                 hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (P < 1 || P > CLSIMG_MAX_P) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pwls_xf_whiten_kernel, dim3(n), dim3(128), 0, st, Li, P, pad_p(P), Flist, n, rowscale, xf);
  return hipGetLastError();
}

// x[i] *= s[i] (mul) or x[i] /= s[i]
__global__ void pwls_scale_kernel(float* __restrict__ x, const float* __restrict__ s, int n, int divide) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    x[i] = divide ? x[i] / s[i] : x[i] * s[i];
}

hipError_t launch_pwls_setup(const float* h, const float* gamma, double C, double kd_coef, int Q, float* rowscale,
                             float* gamma_pw, float* eps_pw, float* dinv, hipStream_t st) {
  const int g = std::min((Q + 255) / 256, 2048);
  hipLaunchKernelGGL(pwls_setup_kernel, dim3(g), dim3(256), 0, st, h, gamma, C, kd_coef, Q, rowscale, gamma_pw,
                     eps_pw, dinv);
  return hipGetLastError();
}

hipError_t launch_pwls_whiten(const double2* Li, const float2* B0, int P, float2* Lw, float2* B0w, hipStream_t st) {
  if (P > 48) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pwls_whiten_kernel, dim3(1), dim3(1024), 0, st, Li, B0, P, Lw, B0w);
  return hipGetLastError();
}

hipError_t launch_pwls_scale(float* x, const float* s, int n, bool divide, hipStream_t st) {
  const int g = std::min((n + 255) / 256, 2048);
  hipLaunchKernelGGL(pwls_scale_kernel, dim3(g), dim3(256), 0, st, x, s, n, divide ? 1 : 0);
  return hipGetLastError();
}

bool outer_fits(int P) { return pad_p(P) / 8 <= 6; }

hipError_t launch_request_init_batch(const ReqInitItem* items, int nreq, int Qmax, hipStream_t s) {
  const int per = std::max(1, std::min(16, (Qmax + 1023) / 1024));
  hipLaunchKernelGGL(request_init_batch_kernel, dim3(nreq * per), dim3(256), 0, s, items, per);
  return hipGetLastError();
}

hipError_t launch_outer_init(OuterState* st, const SolveDecision* dec, hipStream_t s) {
  hipLaunchKernelGGL(outer_init_kernel, dim3(1), dim3(64), 0, s, st, dec);
  return hipGetLastError();
}

// the outer states of a batch, each in its request's slice, into one array
// (one read-back per poll)
static_assert(sizeof(OuterState) % 4 == 0, "the state is copied as 32-bit words");
__global__ void gather_states_kernel(const OuterParams* __restrict__ prs, int n, OuterState* __restrict__ out) {
  constexpr int NW = sizeof(OuterState) / 4;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * NW; e += gridDim.x * blockDim.x) {
    const int r = e / NW, k = e - r * NW;
    reinterpret_cast<int*>(out + r)[k] = reinterpret_cast<const int*>(prs[r].st)[k];
  }
}

hipError_t launch_gather_states(const OuterParams* prs, int n, OuterState* out, hipStream_t s) {
  const int NW = (int)(sizeof(OuterState) / 4);
  const int g = std::min((n * NW + 255) / 256, 1024);
  hipLaunchKernelGGL(gather_states_kernel, dim3(g), dim3(256), 0, s, prs, n, out);
  return hipGetLastError();
}

hipError_t launch_outer_step_batch(const OuterParams* prs, int nreq, int P, hipStream_t s) {
  const dim3 g(nreq), b(kCuThreads);
  switch (pad_p(P) / 8) {
    case 1: hipLaunchKernelGGL(outer_step_batch_kernel<1>, g, b, 0, s, prs); break;
    case 2: hipLaunchKernelGGL(outer_step_batch_kernel<2>, g, b, 0, s, prs); break;
    case 3: hipLaunchKernelGGL(outer_step_batch_kernel<3>, g, b, 0, s, prs); break;
    case 4: hipLaunchKernelGGL(outer_step_batch_kernel<4>, g, b, 0, s, prs); break;
    case 5: hipLaunchKernelGGL(outer_step_batch_kernel<5>, g, b, 0, s, prs); break;
    case 6: hipLaunchKernelGGL(outer_step_batch_kernel<6>, g, b, 0, s, prs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_outer_step(const OuterParams& pr, hipStream_t s) {
  const dim3 g(1), b(kCuThreads);
  switch (pad_p(pr.P) / 8) {
    case 1: hipLaunchKernelGGL(outer_step_kernel<1>, g, b, 0, s, pr); break;
    case 2: hipLaunchKernelGGL(outer_step_kernel<2>, g, b, 0, s, pr); break;
    case 3: hipLaunchKernelGGL(outer_step_kernel<3>, g, b, 0, s, pr); break;
    case 4: hipLaunchKernelGGL(outer_step_kernel<4>, g, b, 0, s, pr); break;
    case 5: hipLaunchKernelGGL(outer_step_kernel<5>, g, b, 0, s, pr); break;
    case 6: hipLaunchKernelGGL(outer_step_kernel<6>, g, b, 0, s, pr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace clsimg
