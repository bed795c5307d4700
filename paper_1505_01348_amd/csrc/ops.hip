// Khatri-Rao operator kernels: beamforming (Psi^H), correlation (Psi), their
// reduction, the real-embedding fragments, and the FP64 Cholesky inverse.
//
// Sec. IV-B of the paper observes that Psi v is a correlation matrix
// sum_i v_i a_i a_i^H and Psi^H u a set of beamformer outputs a_i^H U a_i, so
// that the Khatri-Rao matrix never has to be stored.  Here both become dense
// real GEMMs on the fp32 MFMA with the steering vectors generated on the fly
// from FP64-built separable tables (layout notes in common.h).
#include <algorithm>

#include "kernels.h"

namespace clsimg {

// ---------------------------------------------------------------------------
// Beamforming: g_k = x_k^T Ut x_k for the pixels of a list (or 0..n-1).
// Y = Ut X on MFMA.  Per K-chunk the workgroup stages Ut (A operands, kept
// resident across tiles when it fits) and the steering entries of its T
// pixels (B operands) in LDS, so that every global load of a chunk is in
// flight at once; then a column dot product of Y with X.
constexpr int kLdsU = 12288;     // 48 KiB of Ut per workgroup
constexpr int kMaxKch = 24;      // k-steps per chunk (96 real rows of X)
constexpr int kXsRows = 4 * kMaxKch;

__host__ __device__ inline int adjoint_kch(int MT, int KS) {
  int k = kLdsU / (MT * 64);
  k = k < KS ? k : KS;
  return k < kMaxKch ? k : kMaxKch;
}

template <int MTW, int NTW, int WM, class Epi>
__global__ __launch_bounds__(kThreads) void adjoint_kernel(AdjParams pr, Epi epi) {
  const int stop = pr.stop_flag ? *pr.stop_flag : 0;
  const typename Epi::Ctx cx = epi.init();  // per-block constants of the epilogue
  if (stop) return;
  constexpr int WN = 4 / WM;
  constexpr int T = WN * NTW * 16;
  constexpr int TS = T + 16;  // padded row stride of the staged X (bank spread)
  static_assert(T <= kThreads, "tile wider than the block");
  __shared__ float lds[kLdsU];
  __shared__ float xs[kXsRows * TS];
  __shared__ float gsh[WM][T];
  __shared__ int spix[T];
  __shared__ int sil[T], sim[T];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wm = w % WM, wn = w / WM;
  const int c16 = lane & 15, q = lane >> 4;
  // row tiles held in LDS: MTA = WM*MTW >= MT, the ones past MT are zero so
  // that the MFMA loop carries no branch
  constexpr int MTA = WM * MTW;
  const int MT = pr.MT, KS = pr.KS;
  const int kch = adjoint_kch(MTA, KS);
  const bool resident = (kch == KS);
  const int ntiles = (pr.n + T - 1) / T;
  const Tables tab = pr.tab;
  bool loaded = false;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();
    if (tid < T) {
      const int col = tile * T + tid;
      int pix = -1;
      if (col < pr.n) {
        pix = pr.idx ? pr.idx[col] : col;
        if ((unsigned)pix >= (unsigned)tab.Q) pix = -1;
      }
      spix[tid] = pix;
      const int pp = pix < 0 ? 0 : pix;
      const int im = pp / tab.nl;
      sil[tid] = pp - im * tab.nl;
      sim[tid] = im;
    }
    const int ecol = tile * T + tid;
    const typename Epi::Pre pf = epi.prefetch(ecol, tid < T && ecol < pr.n);
    float gp[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) gp[t] = 0.f;
    // covariance blocks: the column dots of every block add up (one block
    // unless the caller stacks several); Ut of each block is staged anew
    const int kb0 = pr.blk_grid ? (int)blockIdx.y : 0, kb1 = pr.blk_grid ? kb0 + 1 : pr.nblk;
    for (int kb = kb0; kb < kb1; ++kb) {
    const float* fragk = pr.frag ? pr.frag + kb * pr.frag_stride : nullptr;
    Tables tabk = tab;
    tabk.El += kb * pr.tab_stride;
    tabk.Em += kb * pr.tab_stride;
    if (kb1 - kb0 > 1) loaded = false;
    v4f acc[MTW][NTW];
#pragma unroll
    for (int mi = 0; mi < MTW; ++mi)
#pragma unroll
      for (int t = 0; t < NTW; ++t) acc[mi][t] = v4f{0.f, 0.f, 0.f, 0.f};

    for (int kc0 = 0; kc0 < KS; kc0 += kch) {
      const int kn = min(kch, KS - kc0);
      __syncthreads();
      if (!(resident && loaded)) {
        if (pr.U) {
          // stage Ut straight from the complex matrix: Ut[2p+s][2q+u]
          // wave w fills blocks (mt, j) = w, w+4, ...; the lane is the fragment slot
          const int l = lane, s = l & 1, u = (l >> 4) & 1;
          int mt = 0, j = w;
          while (j >= kn) {
            j -= kn;
            ++mt;
          }
          for (; mt < MTA;) {
            const int p = 8 * mt + ((l & 15) >> 1), qq = 2 * (kc0 + j) + (l >> 5);
            const float2 v = (mt < MT && p < pr.P && qq < pr.P) ? pr.U[p * pr.P + qq]
                                                                 : make_float2(0.f, 0.f);
            lds[(mt * kch + j) * 64 + l] = (s == u) ? v.x : (s == 0 ? -v.y : v.y);
            j += 4;
            while (j >= kn) {
              j -= kn;
              ++mt;
            }
          }
        } else {
          const int n4 = MTA * kn * 16;
          for (int e = tid; e < n4; e += kThreads) {
            const int mt = e / (kn * 16);
            const int r = e - mt * kn * 16;
            const int j = r >> 4, l4 = r & 15;
            float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
            if (mt < MT)
              val = *reinterpret_cast<const float4*>(fragk + ((size_t)(mt * KS + kc0 + j) * 64 + l4 * 4));
            *reinterpret_cast<float4*>(lds + ((mt * kch + j) * 64 + l4 * 4)) = val;
          }
        }
        loaded = true;
      }
      // steering entries of antennas 2kc0 .. 2(kc0+kn)-1 for the T pixels
      const int na = 2 * kn;
      if (pr.xf) {
        const int nr = 2 * na, ldx = 2 * tab.Pp;
        for (int e = tid; e < nr * T; e += kThreads) {
          const int c = e / nr, row = e - c * nr;
          const int col = tile * T + c;
          xs[row * TS + c] = (spix[c] >= 0) ? pr.xf[(size_t)col * ldx + 4 * kc0 + row] : 0.f;
        }
      } else {
        for (int e = tid; e < na * T; e += kThreads) {
          const int pl = e / T, c = e - pl * T;  // T is a power of two
          float2 a = make_float2(0.f, 0.f);
          if (spix[c] >= 0) a = tabk.a(2 * kc0 + pl, sil[c], sim[c]);
          xs[(2 * pl) * TS + c] = a.x;
          xs[(2 * pl + 1) * TS + c] = a.y;
        }
      }
      __syncthreads();
#pragma unroll 2
      for (int j = 0; j < kn; ++j) {
        float b[NTW];
#pragma unroll
        for (int t = 0; t < NTW; ++t) b[t] = xs[(4 * j + q) * TS + (wn * NTW + t) * 16 + c16];
        float av[MTW];
#pragma unroll
        for (int mi = 0; mi < MTW; ++mi) av[mi] = lds[((wm * MTW + mi) * kch + j) * 64 + lane];
#pragma unroll
        for (int mi = 0; mi < MTW; ++mi)
#pragma unroll
          for (int t = 0; t < NTW; ++t) acc[mi][t] = mfma16x16x4(av[mi], b[t], acc[mi][t]);
      }
    }
    // column dot product: row 16mt + 4q + r of X against the same row of Y
#pragma unroll
    for (int mi = 0; mi < MTW; ++mi) {
      const int mt = wm * MTW + mi;
      if (mt < MT) {
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
          const int cl = (wn * NTW + t) * 16 + c16;
          float x0, x1, x2, x3;
          if (resident) {
            const int r0 = 16 * mt + 4 * q;
            x0 = xs[(r0 + 0) * TS + cl];
            x1 = xs[(r0 + 1) * TS + cl];
            x2 = xs[(r0 + 2) * TS + cl];
            x3 = xs[(r0 + 3) * TS + cl];
          } else if (pr.xf) {
            const float* xr = pr.xf + (size_t)(tile * T + cl) * 2 * tab.Pp + 16 * mt + 4 * q;
            const bool v = spix[cl] >= 0;
            x0 = v ? xr[0] : 0.f;
            x1 = v ? xr[1] : 0.f;
            x2 = v ? xr[2] : 0.f;
            x3 = v ? xr[3] : 0.f;
          } else {
            const int pix = spix[cl];
            float2 a0 = make_float2(0.f, 0.f), a1 = a0;
            if (pix >= 0) {
              const int il = pix % tab.nl, im = pix / tab.nl;
              a0 = tabk.a(8 * mt + 2 * q, il, im);
              a1 = tabk.a(8 * mt + 2 * q + 1, il, im);
            }
            x0 = a0.x; x1 = a0.y; x2 = a1.x; x3 = a1.y;
          }
          gp[t] += x0 * acc[mi][t][0] + x1 * acc[mi][t][1] + x2 * acc[mi][t][2] + x3 * acc[mi][t][3];
        }
      }
    }
    }  // covariance blocks
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
      gp[t] += __shfl_xor(gp[t], 16, 64);
      gp[t] += __shfl_xor(gp[t], 32, 64);
    }
    __syncthreads();
    if (q == 0) {
#pragma unroll
      for (int t = 0; t < NTW; ++t) gsh[wm][(wn * NTW + t) * 16 + c16] = gp[t];
    }
    __syncthreads();
    const int col = tile * T + tid;
    float g = 0.f;
    bool ok = false;
    int pix = 0;
    if (tid < T) {
#pragma unroll
      for (int k = 0; k < WM; ++k) g += gsh[k][tid];
      ok = col < pr.n;
      if (ok) {
        pix = spix[tid];
        if (pix < 0) {  // invalid pixel index: NaN output
          pix = 0;
          g = __builtin_nanf("");
        }
      }
    }
    epi(tile, col, pix, g, ok, cx, pf);
  }
}

// ---------------------------------------------------------------------------
// Beamforming of a pixel list for arrays beyond 12 row tiles, rows and K
// split over workgroups.  Workgroup (x, y, z) takes NT 16-pixel tiles of the
// list, the row tiles 4y .. 4y + 3 of Ut (one per wave, fragments prepared by
// the correlation) and the z-th of gridDim.z slices of the K chunks, with the
// next chunk's fragment and table loads issued before the current chunk's
// MFMA.  The column dot is linear in Y, so x_m^T (Ut_m,slice x_slice) summed
// over slices and row tiles is the beamformer output: each workgroup leaves
// its partial in part[(z * gridDim.y + y) * n + k], and
// adjoint_rows_finish_kernel adds the partials in that order and applies the
// epilogue.  Embedding as in the
// reduction's fragments: real row 2p + s is component s of antenna p.
template <int NT>
__global__ __launch_bounds__(kThreads) void adjoint_rows_kernel(AdjParams pr, float* __restrict__ part) {
  __shared__ float gs[4][NT * 16];
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4, w = threadIdx.x >> 6;
  const int MT = pr.MT, KS = pr.KS, stride = pr.n;  // partials: one row of pr.n per (slice, row group)
  // the flags, the list length and the first group's pixels in one round trip
  const int stop = pr.stop_flag ? *pr.stop_flag : 0;
  const int ndev = pr.n_dev ? *pr.n_dev : pr.n;
  int pix0[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = max(0, min(16 * (blockIdx.x * NT + t) + c16, pr.n - 1));
    pix0[t] = (pr.idx && pr.n > 0) ? pr.idx[col] : col;
  }
  if (stop) return;
  const int n = min(ndev, pr.n);
  const int mt = 4 * blockIdx.y + w;
  const bool live_row = mt < MT;
  const int mtc = live_row ? mt : MT - 1;  // loads stay in bounds; the dot leaves it out
  const Tables tab = pr.tab;
  const size_t sl = (size_t)2 * tab.nl, sm = (size_t)2 * tab.nm;  // two antennas per chunk
  const int per = (KS + gridDim.z - 1) / gridDim.z;
  const int k0 = blockIdx.z * per, k1 = min(KS, k0 + per);
  const float* fw = pr.frag + (size_t)mtc * KS * 64 + lane;
  // groups of NT 16-pixel tiles, strided over gridDim.x (a list built on the
  // device may be shorter than the launch assumed)
  for (int xb = blockIdx.x; 16 * xb * NT < n; xb += gridDim.x) {
    int il[NT], im[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = 16 * (xb * NT + t) + c16;
      int pix = col < n ? (xb == (int)blockIdx.x ? pix0[t] : (pr.idx ? pr.idx[col] : col)) : 0;
      if ((unsigned)pix >= (unsigned)tab.Q) pix = 0;
      im[t] = pix / tab.nl;
      il[t] = pix - im[t] * tab.nl;
    }
    // the column dot's steering entries (antennas 8mt + 2q, 8mt + 2q + 1), loaded with the K loop's
    float2 ad0[NT], ad1[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int pa = 8 * mtc + 2 * q;
      ad0[t] = tab.a(pa, il[t], im[t]);
      ad1[t] = tab.a(pa + 1, il[t], im[t]);
    }
    // B operand of chunk kc: real row 4kc + q = component q & 1 of antenna 2kc + (q >> 1)
    const float2* elp[NT];
    const float2* emp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      elp[t] = tab.El + (size_t)(q >> 1) * tab.nl + il[t];
      emp[t] = tab.Em + (size_t)(q >> 1) * tab.nm + im[t];
    }
    v4f acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    constexpr int KALL = 24;  // one tile and a short slice: every load of the slice issued at once
    if (NT == 1 && k1 - k0 <= KALL) {
      float fa[KALL];
      float2 te[KALL], tm[KALL];
#pragma unroll
      for (int j = 0; j < KALL; ++j)
        if (k0 + j < k1) {
          fa[j] = fw[(size_t)(k0 + j) * 64];
          te[j] = elp[0][(k0 + j) * sl];
          tm[j] = emp[0][(k0 + j) * sm];
        }
#pragma unroll
      for (int j = 0; j < KALL; ++j)
        if (k0 + j < k1) {
          const float2 x = cmul(te[j], tm[j]);
          acc[0] = mfma16x16x4(fa[j], (q & 1) ? x.y : x.x, acc[0]);
        }
    } else {
      const int kf = k0 < k1 ? k0 : 0;
      float fa = fw[(size_t)kf * 64];
      float2 te[NT], tm[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        te[t] = elp[t][kf * sl];
        tm[t] = emp[t][kf * sm];
      }
      for (int kc = k0; kc < k1; ++kc) {
        const float a = fa;
        float b[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const float2 x = cmul(te[t], tm[t]);
          b[t] = (q & 1) ? x.y : x.x;
        }
        const int kn = kc + 1 < k1 ? kc + 1 : kc;
        fa = fw[(size_t)kn * 64];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          te[t] = elp[t][kn * sl];
          tm[t] = emp[t][kn * sm];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma16x16x4(a, b[t], acc[t]);
      }
    }
    // accumulator element r of lane (c16, q): real row 16mt + 4q + r, i.e.
    // antenna 8mt + 2q + (r >> 1), component r & 1
    float gp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      gp[t] = 0.f;
      if (live_row) {
        const float2 a0 = ad0[t], a1 = ad1[t];
        gp[t] = acc[t][0] * a0.x + acc[t][1] * a0.y + acc[t][2] * a1.x + acc[t][3] * a1.y;
      }
      gp[t] += __shfl_xor(gp[t], 16, 64);
      gp[t] += __shfl_xor(gp[t], 32, 64);
    }
    if (q == 0) {
#pragma unroll
      for (int t = 0; t < NT; ++t) gs[w][16 * t + c16] = gp[t];
    }
    __syncthreads();
    if (threadIdx.x < NT * 16) {
      const int col = 16 * xb * NT + threadIdx.x;
      const float g = (gs[0][threadIdx.x] + gs[1][threadIdx.x]) + (gs[2][threadIdx.x] + gs[3][threadIdx.x]);
      if (col < n) part[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * stride + col] = g;
    }
    __syncthreads();
  }
}

// The row groups' partial dots added in group order, then the epilogue on
// tiles of T <= 64 listed pixels (the tiles of adjoint_kernel), one wave each.
template <class Epi>
__global__ __launch_bounds__(64) void adjoint_rows_finish_kernel(AdjParams pr, const float* __restrict__ part,
                                                                 int ngroups, int T, Epi epi) {
  const int stop = pr.stop_flag ? *pr.stop_flag : 0;
  const int tile = blockIdx.x, col = tile * T + threadIdx.x;
  // the epilogue's inputs with the flag (columns below the host's bound are
  // in bounds; a device-length list's epilogues load nothing here)
  const typename Epi::Pre pf = epi.prefetch(col, (int)threadIdx.x < T && col < pr.n);
  const typename Epi::Ctx cx = epi.init();
  if (stop) return;
  const int n = pr.n_dev ? min(*pr.n_dev, pr.n) : pr.n;
  const bool ok = (int)threadIdx.x < T && col < n;
  float g = 0.f;
  int pix = 0;
  if (ok) {
    // eight partials loaded at a time, added in group order
    int y = 0;
    for (; y + 8 <= ngroups; y += 8) {
      float v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = part[(size_t)(y + k) * pr.n + col];
#pragma unroll
      for (int k = 0; k < 8; ++k) g += v[k];
    }
    for (; y < ngroups; ++y) g += part[(size_t)y * pr.n + col];
    pix = pr.idx ? pr.idx[col] : col;
    if ((unsigned)pix >= (unsigned)pr.tab.Q) {  // invalid pixel index: NaN output
      pix = 0;
      g = __builtin_nanf("");
    }
  }
  epi(tile, col, pix, g, ok, cx, pf);
}

// ---------------------------------------------------------------------------
// Beamforming of a free list for 7..12 row tiles (LSQR adjoint,
// v_raw = Psi_F^H u / beta - beta v with the ||v_raw||^2 partial of the
// tile): one 16-pixel tile per workgroup of MT waves, wave m taking row tile
// m over the whole K.  A wave may hold at most 63 loads in flight, so each
// issues only its KS fragment loads (Ut fragments prepared by the
// correlation) and one float4 of the tile's 16 columns of X_F, which the
// workgroup stages in LDS; the K loop then waits on one round trip to memory.
// The waves' column dots meet in LDS, and wave 0 adds them in row-tile order
// and runs the epilogue alone (wave sums on the VALU, no further barrier).
constexpr int kListThreads = 768;

template <int MT>
__global__ __launch_bounds__(kListThreads) void adjoint_list_kernel(AdjParams pr, EpiLsqrV2 epi) {
  constexpr int KS = 4 * MT, Pp = 8 * MT, RS = 2 * Pp + 4;  // LDS row stride: 2-way banks at most
  constexpr int kBetaPre = 2;  // ||u||^2 partials per lane of wave 0 loaded at launch
  __shared__ float xs[16 * RS];
  __shared__ float gsh[MT][16];
  const int tid = threadIdx.x, lane = tid & 63, m = tid >> 6;
  const int c16 = lane & 15, q = lane >> 4;
  const int tile = blockIdx.x, n = pr.n;
  const int col = 16 * tile + lane;
  // the stop flag, every operand and the epilogue's inputs are requested
  // together (all in bounds whether or not the flag is set)
  const int stop = pr.stop_flag ? *pr.stop_flag : 0;
  const float* fm = pr.frag + (size_t)m * KS * 64 + lane;
  float a[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) a[k] = fm[k * 64];
  {  // 16 columns x 2Pp floats = 64 MT float4s: one per thread
    const int r = tid / (Pp / 2), j = tid - r * (Pp / 2);
    const float4 x = *reinterpret_cast<const float4*>(pr.xf + (size_t)min(16 * tile + r, n - 1) * 2 * Pp + 4 * j);
    float* d = xs + r * RS + 4 * j;
    d[0] = x.x;
    d[1] = x.y;
    d[2] = x.z;
    d[3] = x.w;
  }
  // wave 0 runs the epilogue: beta_{it+1} from the correlation's partials and
  // v_it of its 16 columns
  double bp[kBetaPre] = {0.0, 0.0};
  float vold = 0.f;
  if (m == 0) {
#pragma unroll
    for (int j = 0; j < kBetaPre; ++j)
      if (lane + 64 * j < epi.nbeta) bp[j] = epi.beta_part[lane + 64 * j];
    if (lane < 16 && col < n && !epi.first) vold = epi.vnorm[col];
  }
  if (stop) return;
  double beta = 0.0;
  if (m == 0) {  // while the other waves' operands arrive
    double b2 = bp[0] + bp[1];
    for (int i = lane + 64 * kBetaPre; i < epi.nbeta; i += 64) b2 += epi.beta_part[i];
    beta = sqrt(wave_sum_dpp_d(b2));
  }
  __syncthreads();  // xs complete
  const float* xc = xs + c16 * RS;
  v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < KS; ++k) acc = mfma16x16x4(a[k], xc[4 * k + q], acc);
  // column dot: accumulator element r is row 16 m + 4 q + r
  const float4 xr = *reinterpret_cast<const float4*>(xc + 16 * m + 4 * q);
  float gp = xr.x * acc[0] + xr.y * acc[1] + xr.z * acc[2] + xr.w * acc[3];
  gp += __shfl_xor(gp, 16, 64);
  gp += __shfl_xor(gp, 32, 64);
  if (q == 0) gsh[m][c16] = gp;
  __syncthreads();
  if (m != 0) return;
  double vr2 = 0.0;
  if (lane < 16 && col < n) {
    float g = 0.f;
#pragma unroll
    for (int i = 0; i < MT; ++i) g += gsh[i][lane];
    const int pix = pr.idx ? pr.idx[col] : col;
    if ((unsigned)pix >= (unsigned)pr.tab.Q) g = __builtin_nanf("");  // invalid pixel index: NaN output
    double vr = beta > 0.0 ? (double)g / beta : 0.0;
    if (!epi.first) vr -= beta * (double)vold;
    const float vf = (float)vr;
    epi.vraw[col] = vf;
    vr2 = (double)vf * vf;
  }
  vr2 = wave_sum_dpp_d(vr2);
  if (lane == 0) epi.alpha_part[tile] = vr2;
}

// ---------------------------------------------------------------------------
// Correlation (forward operator, Sec. IV-B): Y = sum_k v_k a_k a_k^H over a
// pixel list, computed in complex form on 16 x 16 antenna tiles.  For tiles
// (bm, bn) of antennas, per four pixels (one MFMA k step, lane group q = one
// pixel), with A = a[16bm + c16] and B = v a[16bn + c16]:
//   Re Y += A_r B_r + A_i B_i,   Im Y += A_i B_r - A_r B_i,
// four 16x16x4 FP32 MFMAs, exactly the dense complex count (8 flops per term
// and antenna pair); Y is Hermitian, so only tile pairs bm >= bn are formed.
// A wave owns a BT x BT block of tile pairs and generates its 2 BT steering
// entries per pixel straight into registers from the tables (one complex
// product each), with the next step's table entries, pixel indices and
// weights loaded while the current step multiplies.  The four waves of a
// workgroup split the workgroup's pixels (k steps w, w + 4, ...) and their
// accumulators are added in LDS in a fixed order; each workgroup leaves one
// partial of its block pair: part[(chunk * npairs + pair) * BT^2 * 512 +
// tile * 512 + {0: Re, 256: Im} + lane * 4 + r] = Y[16 bm + 4q + r][16 bn + c16].

template <int BT, bool TR, bool LIST>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void corr_kernel(FwdParams pr) {
  constexpr int NACC = BT * BT * 2;  // v4f accumulators per lane: Re and Im of each tile pair
  __shared__ v4f red[2][NACC][64];
  if (pr.stop_flag && *pr.stop_flag) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c16 = lane & 15, q = lane >> 4;
  int BM = 0, BN = blockIdx.y;  // the y-th block pair of (0,0), (1,0), (1,1), (2,0), ...
  while (BN > BM) {
    BN -= BM + 1;
    ++BM;
  }
  const bool diag = BM == BN;
  Tables tab = pr.tab;
  tab.El += blockIdx.z * pr.tab_stride;
  tab.Em += blockIdx.z * pr.tab_stride;
  const int Pp = tab.Pp, nl = tab.nl, nm = tab.nm;
  // this lane's antennas: rows 16 (BT BM + i) + c16, columns 16 (BT BN + j) + c16
  int ar[BT], ac[BT];
#pragma unroll
  for (int i = 0; i < BT; ++i) {
    ar[i] = 16 * (BT * BM + i) + c16;
    ac[i] = 16 * (BT * BN + i) + c16;
  }
  const int k0 = blockIdx.x * pr.chw, k1 = min(k0 + pr.chw, pr.n);
  v4f acc[NACC];
#pragma unroll
  for (int a = 0; a < NACC; ++a) acc[a] = v4f{0.f, 0.f, 0.f, 0.f};
  // pixel of step s for this lane: k = k0 + 16 s + 4 w + q (LIST: the k-th
  // entry of the index list); over the whole grid its (im, il) advance by 16
  // pixels a step, and no load stands between a step's table loads and the
  // next step's
  const bool walk = !LIST && nl >= 16;
  auto pix_of = [&](int k, int& pix, float& v) {
    pix = 0;
    v = 0.f;
    if (k < k1) {
      int p = LIST ? pr.idx[k] : k;
      const bool ok = (unsigned)p < (unsigned)tab.Q;  // invalid index: term dropped
      pix = ok ? p : 0;
      v = ok ? (pr.gather ? pr.vals[pix] : pr.vals[k]) : 0.f;
    }
  };
  float2 elr[BT], emr[BT], elc[BT], emc[BT];
  // TR: antenna-fastest tables with rows of corr_rows(Pp) entries, zero
  // beyond P (a lane group's 16 antennas of a pixel are contiguous, fixed
  // offsets from one base per lane, no bounds test); else pixel-fastest
  const int rowT = corr_rows(Pp);
  auto fetch = [&](int im, int il) {
    if (TR) {
      // one base per table and block side; tile i at a fixed offset of 16 i entries
      const float2* lr = tab.ElT + ((size_t)il * rowT + (size_t)ar[0]);
      const float2* mr = tab.EmT + ((size_t)im * rowT + (size_t)ar[0]);
      const float2* lc = tab.ElT + ((size_t)il * rowT + (size_t)ac[0]);
      const float2* mc = tab.EmT + ((size_t)im * rowT + (size_t)ac[0]);
#pragma unroll
      for (int i = 0; i < BT; ++i) {
        elr[i] = lr[16 * i];
        emr[i] = mr[16 * i];
        if (!diag) {
          elc[i] = lc[16 * i];
          emc[i] = mc[16 * i];
        }
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < BT; ++i) {
      const bool okr = ar[i] < Pp, okc = ac[i] < Pp;
      elr[i] = okr ? tab.El[(size_t)ar[i] * nl + il] : make_float2(0.f, 0.f);
      emr[i] = okr ? tab.Em[(size_t)ar[i] * nm + im] : make_float2(0.f, 0.f);
      if (!diag) {
        elc[i] = okc ? tab.El[(size_t)ac[i] * nl + il] : make_float2(0.f, 0.f);
        emc[i] = okc ? tab.Em[(size_t)ac[i] * nm + im] : make_float2(0.f, 0.f);
      }
    }
  };
  int kk = k0 + 4 * w + q;
  int pix;
  float v;
  pix_of(kk, pix, v);
  int im = pix / nl, il = pix - im * nl;
  fetch(im, il);
  for (int kb = k0 + 4 * w; kb < k1; kb += 16) {
    float2 A[BT], C[BT];
#pragma unroll
    for (int i = 0; i < BT; ++i) {
      A[i] = cmul(elr[i], emr[i]);
      C[i] = diag ? A[i] : cmul(elc[i], emc[i]);
    }
    const float vc = v;
    // the next step's pixel and table entries
    kk += 16;
    pix_of(kk, pix, v);
    if (walk && kk < k1) {
      il += 16;
      while (il >= nl) {
        il -= nl;
        ++im;
      }
    } else {
      im = pix / nl;
      il = pix - im * nl;
    }
    fetch(im, il);
    float br[BT], bi[BT], bn[BT];
#pragma unroll
    for (int j = 0; j < BT; ++j) {
      br[j] = vc * C[j].x;
      bi[j] = vc * C[j].y;
      bn[j] = -bi[j];
    }
#pragma unroll
    for (int i = 0; i < BT; ++i)
#pragma unroll
      for (int j = 0; j < BT; ++j) {
        if (diag && j > i) continue;  // upper tiles of a diagonal block: mirrors
        v4f& re = acc[2 * (i * BT + j)];
        v4f& im = acc[2 * (i * BT + j) + 1];
        re = mfma16x16x4(A[i].x, br[j], re);
        re = mfma16x16x4(A[i].y, bi[j], re);
        im = mfma16x16x4(A[i].y, br[j], im);
        im = mfma16x16x4(A[i].x, bn[j], im);
      }
  }
  // the four waves' accumulators: (w0 + w2) + (w1 + w3)
  if (w >= 2) {
#pragma unroll
    for (int a = 0; a < NACC; ++a) red[w - 2][a][lane] = acc[a];
  }
  __syncthreads();
  if (w < 2) {
#pragma unroll
    for (int a = 0; a < NACC; ++a) {
      const v4f o = red[w][a][lane];
      acc[a] = v4f{acc[a][0] + o[0], acc[a][1] + o[1], acc[a][2] + o[2], acc[a][3] + o[3]};
    }
  }
  __syncthreads();
  if (w == 1) {
#pragma unroll
    for (int a = 0; a < NACC; ++a) red[0][a][lane] = acc[a];
  }
  __syncthreads();
  if (w == 0) {
    float* part = pr.part + blockIdx.z * pr.part_stride +
                  ((size_t)blockIdx.x * gridDim.y + blockIdx.y) * (size_t)(BT * BT * 512);
#pragma unroll
    for (int a = 0; a < NACC; ++a) {
      const v4f o = red[0][a][lane];
      const float4 r = make_float4(acc[a][0] + o[0], acc[a][1] + o[1], acc[a][2] + o[2], acc[a][3] + o[3]);
      // pair t = a / 2, component a & 1
      *reinterpret_cast<float4*>(part + (size_t)(a >> 1) * 512 + (a & 1) * 256 + lane * 4) = r;
    }
  }
}

// ---------------------------------------------------------------------------
// Second stage of the correlation: one workgroup per antenna tile pair
// (bm >= bn) sums the chunks' partials in chunk order (each thread one entry,
// a fixed order), then writes
//   out = cK * Y + cB * B  (complex P x P; cB may come from the LSQR state,
//   -alpha/beta), at (p, q) and, off the diagonal tile, at (q, p) with
//   Y_qp = conj(Y_pq);
// optionally the Ut fragments of out (interleaved embedding, layout of
// common.h) and the workgroup's sum |out|^2 in norm_part[blockIdx.x].  out may
// alias B.  Partials are read at the block pair and tile of the correlation.
constexpr int kRedGroups = 4;  // thread groups summing interleaved chunks
// The output of one tile pair from its sum y = Y_pq (writer threads only):
// out = cK Y + cB B on the tile's lower part and mirrored, the fragments of
// out, and the workgroup's share of |out|^2 (every thread of the workgroup
// calls it: the norm is a block sum).
// The entries of B this thread's outputs add and the LSQR scalars, requested
// before the kernel's own sums so that they arrive meanwhile.
struct RedPre {
  float2 b[2];  // B[p][q] and B[q][p] of the thread's entry and its mirror
  double alpha, beta;
};

__device__ __forceinline__ RedPre red_prefetch(const RedParams& pr, int bm, int bn, int row, int col, bool writer) {
  RedPre r;
  r.b[0] = r.b[1] = make_float2(0.f, 0.f);
  r.alpha = r.beta = 0.0;
  if (pr.lsqr) {
    r.alpha = pr.lsqr->alpha;
    r.beta = pr.lsqr->beta;
  }
  const int P = pr.P, p = 16 * bm + row, qq = 16 * bn + col;
  if (pr.B && writer && (bm != bn || row >= col) && p < P && qq < P) {
    r.b[0] = pr.B[(size_t)p * P + qq];
    if (p != qq) r.b[1] = pr.B[(size_t)qq * P + p];
  }
  return r;
}

template <int NW>
__device__ __forceinline__ void red_store(const RedParams& pr, int bm, int bn, int row, int col, bool writer,
                                          float yr, float yi, double (&sh)[NW], const RedPre& pre) {
  const int P = pr.P, Pp = pad_p(P);
  const int p = 16 * bm + row, qq = 16 * bn + col;
  float cB = pr.cB;
  if (pr.lsqr) cB = (float)(-pre.alpha / pre.beta);
  // the diagonal tile: its lower triangle, mirrored
  const bool lower = writer && (bm != bn || row >= col);
  double nrm = 0.0;
  const int KS = Pp / 2;
  auto put = [&](int a, int b, float2 y, float2 bv) {  // out[a][b] from Y_ab = y and B[a][b] = bv
    float2 o = make_float2(0.f, 0.f);
    if (a < P && b < P) {
      o = make_float2(pr.cK * y.x, pr.cK * y.y);
      if (pr.B) {
        o.x += cB * bv.x;
        o.y += cB * bv.y;
      }
      pr.out[(size_t)a * P + b] = o;
      nrm += (double)o.x * o.x + (double)o.y * o.y;
    }
    if (pr.frag && a < Pp && b < Pp) {
#pragma unroll
      for (int su = 0; su < 4; ++su) {
        const int s_ = su >> 1, u_ = su & 1;
        const int rr = 2 * a + s_, cc = 2 * b + u_;
        const float fv = (s_ == u_) ? o.x : (s_ == 0 ? -o.y : o.y);
        pr.frag[((size_t)(rr >> 4) * KS + (cc >> 2)) * 64 + (cc & 3) * 16 + (rr & 15)] = fv;
      }
    }
  };
  if (lower) {
    if (p == qq) yi = 0.f;  // the diagonal of a Hermitian matrix is real
    put(p, qq, make_float2(yr, yi), pre.b[0]);
    if (p != qq) put(qq, p, make_float2(yr, -yi), pre.b[1]);
  }
  if (pr.norm_part) {
    const double tot = block_sum_dpp_d(nrm, sh);
    if (threadIdx.x == 0) pr.norm_part[blockIdx.x] = tot;
  }
}

__device__ __forceinline__ void red_pair(int b, int& bm, int& bn) {  // tile pair b, bm >= bn
  bm = 0;
  bn = b;
  while (bn > bm) {
    bn -= bm + 1;
    ++bm;
  }
}

__global__ __launch_bounds__(256 * kRedGroups) void reduce_kernel(RedParams pr) {
  __shared__ double sh[4 * kRedGroups];
  __shared__ float2 gsum[kRedGroups - 1][256];
  const int stop = pr.stop_flag ? *pr.stop_flag : 0;
  {  // covariance block blockIdx.y
    const size_t kb = blockIdx.y;
    pr.part += kb * pr.part_stride;
    pr.out += kb * pr.out_stride;
    if (pr.B) pr.B += kb * pr.B_stride;
    if (pr.frag) pr.frag += kb * pr.frag_stride;
    if (pr.norm_part) pr.norm_part += kb * pr.norm_stride;
  }
  const int P = pr.P, BT = corr_bt(P), npairs = corr_pairs(P);
  int bm, bn;  // tile pair (bm >= bn)
  red_pair(blockIdx.x, bm, bn);
  const int BM = bm / BT, BN = bn / BT;
  const int pair = BM * (BM + 1) / 2 + BN, tile = (bm - BT * BM) * BT + (bn - BT * BN);
  const int t = threadIdx.x & 255, grp = threadIdx.x >> 8, lane = t >> 2, r = t & 3;
  const int row = 4 * (lane >> 4) + r, col = lane & 15;
  const RedPre pre = red_prefetch(pr, bm, bn, row, col, grp == 0);
  if (stop) return;
  // group g sums chunks g, g + G, ...; the group sums are added in group order
  float yr = 0.f, yi = 0.f;
  for (int c = grp; c < pr.nchunks; c += kRedGroups) {
    const float* src = pr.part + ((size_t)c * npairs + pair) * (size_t)(BT * BT * 512) + (size_t)tile * 512;
    yr += src[t];
    yi += src[256 + t];
  }
  if (grp > 0) gsum[grp - 1][t] = make_float2(yr, yi);
  __syncthreads();
  if (grp == 0) {
#pragma unroll
    for (int g = 0; g < kRedGroups - 1; ++g) {
      yr += gsum[g][t].x;
      yi += gsum[g][t].y;
    }
  }
  // group 0 writes
  red_store(pr, bm, bn, row, col, grp == 0, yr, yi, sh, pre);
}

// The correlation of a short list (n <= kCorrSmall pixels) straight into the
// output: one workgroup per 16 x 16 tile pair (the tiles of reduce_kernel,
// the same output, fragments and norm partials), the list's steering entries
// at the pair's 16 + 16 antennas and its weights staged in LDS, then
// Y_pq = sum_k v_k a_k[p] conj(a_k[q]) by one thread per entry.  No partial
// tiles and no second launch.
constexpr int kCorrSmall = 32;
__global__ __launch_bounds__(256) void corr_small_kernel(FwdParams f, RedParams pr) {
  __shared__ float2 sa[kCorrSmall][32];
  __shared__ float sv[kCorrSmall];
  __shared__ double sh[4];
  const int stop = pr.stop_flag ? *pr.stop_flag : 0;
  const Tables& tab = f.tab;
  const int Pp = pad_p(pr.P), n = f.n;
  int bm, bn;
  red_pair(blockIdx.x, bm, bn);
  const int t = threadIdx.x, lane = t >> 2, r = t & 3;
  const int row = 4 * (lane >> 4) + r, col = lane & 15;
  const RedPre pre = red_prefetch(pr, bm, bn, row, col, true);
  // n x 32 steering entries, kSmallIt per thread: every pixel index first,
  // then every table entry and weight, so the staging waits on two round
  // trips to memory instead of two per entry
  constexpr int kSmallIt = kCorrSmall * 32 / 256;
  int pix[kSmallIt];
#pragma unroll
  for (int i = 0; i < kSmallIt; ++i) {
    const int e = t + 256 * i, k = e >> 5;
    int p = 0;
    if (e < n * 32) p = f.idx ? f.idx[k] : k;
    pix[i] = (unsigned)p < (unsigned)tab.Q ? p : 0;  // an invalid index reads in bounds
  }
  int vpix = 0;
  if (t < n) {
    vpix = f.idx ? f.idx[t] : t;
    if ((unsigned)vpix >= (unsigned)tab.Q) vpix = 0;
  }
  float2 el[kSmallIt], em[kSmallIt];
#pragma unroll
  for (int i = 0; i < kSmallIt; ++i) {
    const int e = t + 256 * i, j = e & 31;
    const int ant = min(j < 16 ? 16 * bm + j : 16 * bn + j - 16, Pp - 1);
    const int im = pix[i] / tab.nl;
    el[i] = tab.El[ant * tab.nl + (pix[i] - im * tab.nl)];
    em[i] = tab.Em[ant * tab.nm + im];
  }
  float wv = 0.f;
  if (t < n) wv = f.gather ? f.vals[vpix] : f.vals[t];
#pragma unroll
  for (int i = 0; i < kSmallIt; ++i) {
    const int e = t + 256 * i;
    if (e < n * 32) sa[e >> 5][e & 31] = cmul(el[i], em[i]);
  }
  if (stop) return;
  if (t < n) sv[t] = wv;
  __syncthreads();
  float yr = 0.f, yi = 0.f;
  for (int k = 0; k < n; ++k) {
    const float2 a = sa[k][row], b = sa[k][16 + col];
    const float v = sv[k];
    yr += v * (a.x * b.x + a.y * b.y);
    yi += v * (a.y * b.x - a.x * b.y);
  }
  red_store(pr, bm, bn, row, col, true, yr, yi, sh, pre);
}

// ---------------------------------------------------------------------------
// FP64 Cholesky R = L L^H for arrays beyond the LDS-resident kernel below:
// a blocked right-looking factorisation in panels of kCholNB columns.  W holds
// L row-major, LT its transpose, D the inverses D_b of the diagonal blocks
// L_bb (kCholNB x kCholNB row-major, zero above the diagonal and beyond the
// array).  One launch per panel:
//
// chol_convert_kernel (one workgroup): W = R in FP64 and the first diagonal
// block factored (status 2 for a non-finite entry, 1 for a pivot that is not
// positive, else 0).
// chol_update_kernel (panel j; one workgroup per 32 x 32 tile of the trailing
// lower triangle): the panel's rows below its diagonal block,
// L_ij = A_ij L_jj^-H = A_ij D_j^H, formed in LDS for the tile's two row
// blocks (the diagonal tiles record them in LT), then
// W[i][k] -= sum_c L[i][c] conj(L[k][c]) over the panel's columns; the
// workgroup of the first tile, which holds the whole next diagonal block once
// updated, factors it (chol_block) and stores L_bb and D_b.
// chol_lower_kernel: the rows of L below the diagonal blocks copied from LT
// into W (the update launches read the panel's entries of W while it is
// formed, so they do not overwrite them).
// A diagonal block is factored in LDS one column at a time (chol_block); its
// inverse by forward substitution, one thread per column.
//
// chol_solve_kernel (one workgroup per column c of the identity): forward
// substitution L y = e_c by blocks of kCholNB rows (y_i = -D_i sum_k L_ik y_k,
// y = column c of L^-1, stored when Li is given), then backward substitution
// L^H x = y by blocks (x_i = D_i^H (y_i - sum_k L_ki^H x_k), x = column c of
// R^-1, rounded to complex64).  16 threads share each row's sum (coalesced
// reads of a row of L or of LT), and the next block row's entries are loaded
// while one is reduced: two barriers per block row.
constexpr int kCholNB = 16;
constexpr int kCholMaxRows = 288;  // the largest array (CLSIMG_MAX_P)
constexpr int kCholTile = 32;

// Factor the n x n block in a (kCholNB rows of kCholNB + 1, lower triangle)
// in place; rl[c] = 1 / L_cc.  Every thread of the workgroup calls it
// (blockDim >= kCholNB^2, after a barrier that made a visible); false, in
// every thread, for a pivot that is not positive.  Column c's step subtracts
// a[r][c] conj(a[c2][c]) / a[c][c] from the later columns (r >= c2 > c) while
// column c itself stays unscaled, so a step reads only what the previous one
// wrote (one barrier per column); the columns are scaled by 1 / sqrt(pivot) at
// the end.
__device__ __forceinline__ bool chol_block(double2* a, double* rl, int n) {
  constexpr int NB = kCholNB, LDP = NB + 1;
  const int tid = threadIdx.x, r = tid / NB, c2 = tid - r * NB;
  const bool mine = tid < NB * NB && r < n && c2 <= r;
  for (int c = 0; c < n; ++c) {
    const double d = a[c * LDP + c].x;  // the same value in every thread: the exit is uniform
    if (!(d > 0.0)) return false;
    if (mine && c2 > c) {
      const double rd = 1.0 / d;
      const double2 x = a[r * LDP + c], b = a[c2 * LDP + c];
      double2 v = a[r * LDP + c2];
      v.x -= (x.x * b.x + x.y * b.y) * rd;
      v.y -= (x.y * b.x - x.x * b.y) * rd;
      a[r * LDP + c2] = v;
    }
    __syncthreads();
  }
  double2 v = make_double2(0.0, 0.0);
  double ljj = 1.0;
  if (mine) {
    ljj = sqrt(a[c2 * LDP + c2].x);
    v = a[r * LDP + c2];
  }
  __syncthreads();
  if (mine) {
    a[r * LDP + c2] = r == c2 ? make_double2(ljj, 0.0) : make_double2(v.x / ljj, v.y / ljj);
    if (r == c2) rl[c2] = 1.0 / ljj;
  }
  __syncthreads();
  return true;
}

// After chol_block: L_bb to W and LT at (b0, b0), D_b = L_bb^-1 to Db.
__device__ __forceinline__ void chol_block_store(const double2* a, const double* rl, int n, int b0, int P,
                                                 double2* __restrict__ W, double2* __restrict__ LT,
                                                 double2* __restrict__ Db) {
  constexpr int NB = kCholNB, LDP = NB + 1;
  const int tid = threadIdx.x;
  if (tid < NB * NB) {
    const int r = tid / NB, c = tid - r * NB;
    if (r < n && c <= r) {
      const double2 v = a[r * LDP + c];
      W[(size_t)(b0 + r) * P + b0 + c] = v;
      LT[(size_t)(b0 + c) * P + b0 + r] = v;
    }
  }
  if (tid < NB) {  // column cc of the inverse
    const int cc = tid;
    double2 x[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) x[r] = make_double2(r == cc ? 1.0 : 0.0, 0.0);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (k < n) {
        const double q = rl[k];
        x[k] = make_double2(x[k].x * q, x[k].y * q);
#pragma unroll
        for (int r = k + 1; r < NB; ++r) {
          const double2 l = a[r * LDP + k];
          x[r].x -= l.x * x[k].x - l.y * x[k].y;
          x[r].y -= l.x * x[k].y + l.y * x[k].x;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) Db[r * NB + cc] = (r < n && cc < n) ? x[r] : make_double2(0.0, 0.0);
  }
}

__global__ __launch_bounds__(1024) void chol_convert_kernel(const float2* __restrict__ R, int P,
                                                            double2* __restrict__ W, double2* __restrict__ LT,
                                                            double2* __restrict__ D, int* __restrict__ status) {
  constexpr int NB = kCholNB, LDP = NB + 1;
  __shared__ int bad;
  __shared__ double2 a[NB * LDP];
  __shared__ double rl[NB];
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  const int n2 = P * P;
  int e = tid;
  for (; e + 7 * nt < n2; e += 8 * nt) {
    float2 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = R[e + k * nt];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (!isfinite(v[k].x) || !isfinite(v[k].y)) bad = 2;
      W[e + k * nt] = make_double2((double)v[k].x, (double)v[k].y);
    }
  }
  for (; e < n2; e += nt) {
    const float2 v = R[e];
    if (!isfinite(v.x) || !isfinite(v.y)) bad = 2;
    W[e] = make_double2((double)v.x, (double)v.y);
  }
  // the first diagonal block, from R
  const int n = min(NB, P);
  if (tid < NB * NB) {
    const int r = tid / NB, c = tid - r * NB;
    const float2 v = (r < n && c <= r) ? R[r * P + c] : make_float2(0.f, 0.f);
    a[r * LDP + c] = make_double2((double)v.x, (double)v.y);
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) *status = bad;
    return;
  }
  if (!chol_block(a, rl, n)) {
    if (tid == 0) *status = 1;
    return;
  }
  chol_block_store(a, rl, n, 0, P, W, LT, D);
  if (tid == 0) *status = 0;
}

__global__ __launch_bounds__(256) void chol_update_kernel(double2* __restrict__ W, double2* __restrict__ LT,
                                                          double2* __restrict__ D, int P, int j0,
                                                          int* __restrict__ status) {
  constexpr int NB = kCholNB, LDP = NB + 1, T = kCholTile;
  __shared__ double2 ai[T * LDP], ak[T * LDP], li[T * LDP], lk[T * LDP], dj[NB * NB], a[NB * LDP];
  __shared__ double rl[NB];
  const int t0 = j0 + NB;
  // this workgroup's tile (ti, tk), tk <= ti, in row-major order of the lower triangle
  int ti = 0, b = blockIdx.x;
  while (b > ti) {
    b -= ti + 1;
    ++ti;
  }
  const int tk = b;
  const int i0 = t0 + T * ti, k0 = t0 + T * tk;
  const int tid = threadIdx.x;
  // every load at once (256 threads): the status, D_j, the panel's two row
  // blocks and this thread's trailing entries, row i0 + (tid >> 3), columns
  // k0 + (tid & 7) + 8 u; all in bounds whether or not the status is set
  const int st = *status;
  const double2 djv = D[(size_t)(j0 / NB) * NB * NB + tid];  // NB * NB = 256 entries
  constexpr int kPanelIt = T * NB / 256;
  double2 av[kPanelIt], kv[kPanelIt];
#pragma unroll
  for (int it = 0; it < kPanelIt; ++it) {
    const int e = tid + 256 * it, r = e / NB, c = e - r * NB;
    av[it] = i0 + r < P ? W[(size_t)(i0 + r) * P + j0 + c] : make_double2(0.0, 0.0);
    kv[it] = k0 + r < P ? W[(size_t)(k0 + r) * P + j0 + c] : make_double2(0.0, 0.0);
  }
  const int ri = tid >> 3, i = i0 + ri;
  double2 wv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int k = k0 + (tid & 7) + 8 * u;
    wv[u] = (i < P && k <= i) ? W[(size_t)i * P + k] : make_double2(0.0, 0.0);
  }
  if (st != 0) return;
  dj[tid] = djv;
#pragma unroll
  for (int it = 0; it < kPanelIt; ++it) {
    const int e = tid + 256 * it, r = e / NB, c = e - r * NB;
    ai[r * LDP + c] = av[it];
    ak[r * LDP + c] = kv[it];
  }
  __syncthreads();
  // the panel's rows of L: l[r][c] = sum_{c1 <= c} a[r][c1] conj(D_j[c][c1])
  for (int e = tid; e < T * NB; e += blockDim.x) {
    const int r = e / NB, c = e - r * NB;
    double2 si = make_double2(0.0, 0.0), sk = make_double2(0.0, 0.0);
#pragma unroll
    for (int c1 = 0; c1 < NB; ++c1)
      if (c1 <= c) {
        const double2 d = dj[c * NB + c1], x = ai[r * LDP + c1], y = ak[r * LDP + c1];
        si.x += x.x * d.x + x.y * d.y;
        si.y += x.y * d.x - x.x * d.y;
        sk.x += y.x * d.x + y.y * d.y;
        sk.y += y.y * d.x - y.x * d.y;
      }
    li[r * LDP + c] = si;
    lk[r * LDP + c] = sk;
  }
  __syncthreads();
  if (ti == tk)  // the tile's rows of the panel, recorded transposed
    for (int e = tid; e < T * NB; e += blockDim.x) {
      const int c = e / T, r = e - c * T;
      if (i0 + r < P) LT[(size_t)(j0 + c) * P + i0 + r] = li[r * LDP + c];
    }
  double2 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = make_double2(0.0, 0.0);
#pragma unroll 4
  for (int c = 0; c < NB; ++c) {
    const double2 x = li[ri * LDP + c];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double2 y = lk[((tid & 7) + 8 * u) * LDP + c];
      acc[u].x += x.x * y.x + x.y * y.y;
      acc[u].y += x.y * y.x - x.x * y.y;
    }
  }
  const bool first = ti == 0 && tk == 0;  // holds the next diagonal block (rows and columns t0 .. t0 + NB - 1)
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int kc = (tid & 7) + 8 * u, k = k0 + kc;
    const double2 v = make_double2(wv[u].x - acc[u].x, wv[u].y - acc[u].y);
    if (first && ri < NB && kc < NB)
      a[ri * LDP + kc] = (i < P && k <= i) ? v : make_double2(0.0, 0.0);
    else if (i < P && k <= i)
      W[(size_t)i * P + k] = v;
  }
  if (first) {
    const int n = min(NB, P - t0);
    __syncthreads();
    if (!chol_block(a, rl, n)) {
      if (tid == 0) *status = 1;
      return;
    }
    chol_block_store(a, rl, n, t0, P, W, LT, D + (size_t)(t0 / NB) * NB * NB);
  }
}

__global__ __launch_bounds__(256) void chol_lower_kernel(double2* __restrict__ W, const double2* __restrict__ LT,
                                                         int P, const int* __restrict__ status) {
  constexpr int NB = kCholNB;
  if (*status != 0) return;
  const int bi = blockIdx.x + 1, r0 = bi * NB, n = min(NB, P - r0);
  for (int e = threadIdx.x; e < r0 * NB; e += blockDim.x) {
    const int k = e / NB, r = e - k * NB;
    if (r < n) W[(size_t)(r0 + r) * P + k] = LT[(size_t)k * P + r0 + r];
  }
}

// sum over the 16 lanes of a row group (lanes 16 g .. 16 g + 15 of a wave)
__device__ inline double2 chol_sum16(double2 v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 16);
    v.y += __shfl_xor(v.y, o, 16);
  }
  return v;
}

__global__ __launch_bounds__(256) void chol_solve_kernel(const double2* __restrict__ L, const double2* __restrict__ LT,
                                                         const double2* __restrict__ D, int P,
                                                         const int* __restrict__ status, double2* __restrict__ Li,
                                                         float2* __restrict__ Rinv) {
  constexpr int NB = kCholNB, MB = kCholMaxRows / kCholNB;
  __shared__ double2 y[kCholMaxRows];
  __shared__ double2 t[NB];
  if (*status != 0) return;
  const int c = blockIdx.x, tid = threadIdx.x, r = tid >> 4, q = tid & 15;
  const int nbk = (P + NB - 1) / NB, jc = c / NB;
  // block jc of y: column (c - NB jc) of D_jc; above it zero
  for (int i = tid; i < nbk * NB; i += blockDim.x)
    y[i] = i / NB == jc ? D[(size_t)jc * NB * NB + (i - jc * NB) * NB + (c - jc * NB)] : make_double2(0.0, 0.0);
  // forward, block rows i > jc: y_i = -D_i sum_{k in blocks jc .. i-1} L_ik y_k.  Thread (r, q) sums
  // L[i NB + r][jc NB + q + NB m] y[jc NB + q + NB m] over m; the next block row's entries are
  // loaded while this one is reduced.
  double2 nxt[MB];
  auto load_fwd = [&](int i) {
    const int row = i * NB + r, cnt = i - jc;
    const double2* lr = L + (size_t)min(row, P - 1) * P + jc * NB + q;
#pragma unroll
    for (int m = 0; m < MB; ++m) nxt[m] = (m < cnt && row < P) ? lr[m * NB] : make_double2(0.0, 0.0);
  };
  if (jc + 1 < nbk) load_fwd(jc + 1);
  __syncthreads();
  for (int i = jc + 1; i < nbk; ++i) {
    double2 lv[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) lv[m] = nxt[m];
    if (i + 1 < nbk) load_fwd(i + 1);
    const int cnt = i - jc;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int m = 0; m < MB; ++m)
      if (m < cnt) {
        const double2 v = y[jc * NB + q + m * NB];
        acc.x += lv[m].x * v.x - lv[m].y * v.y;
        acc.y += lv[m].x * v.y + lv[m].y * v.x;
      }
    acc = chol_sum16(acc);
    if (q == 0) t[r] = make_double2(-acc.x, -acc.y);
    __syncthreads();
    const double2 d = D[(size_t)i * NB * NB + r * NB + q], tq = t[q];
    double2 p = make_double2(d.x * tq.x - d.y * tq.y, d.x * tq.y + d.y * tq.x);
    p = chol_sum16(p);
    if (q == 0) y[i * NB + r] = p;
    __syncthreads();
  }
  if (Li)
    for (int i = tid; i < P; i += blockDim.x) Li[(size_t)i * P + c] = y[i];
  // backward, block rows i = nbk-1 .. 0: x_i = D_i^H (y_i - sum_{k >= (i+1) NB} conj(L_ki) x_k), x
  // overwriting y; conj(L[k][i NB + r]) is entry k of row i NB + r of LT
  auto load_bwd = [&](int i) {
    const int row = i * NB + r, k0 = (i + 1) * NB + q;
    const double2* lr = LT + (size_t)min(row, P - 1) * P;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int k = k0 + m * NB;
      nxt[m] = (k < P && row < P) ? lr[k] : make_double2(0.0, 0.0);
    }
  };
  load_bwd(nbk - 1);
  for (int i = nbk - 1; i >= 0; --i) {
    double2 lv[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) lv[m] = nxt[m];
    if (i > 0) load_bwd(i - 1);
    const int k0 = (i + 1) * NB + q;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      const int k = k0 + m * NB;
      if (k < P) {
        const double2 v = y[k];  // conj(l) v
        acc.x += lv[m].x * v.x + lv[m].y * v.y;
        acc.y += lv[m].x * v.y - lv[m].y * v.x;
      }
    }
    acc = chol_sum16(acc);
    if (q == 0) {
      const double2 yi = y[i * NB + r];
      t[r] = make_double2(yi.x - acc.x, yi.y - acc.y);
    }
    __syncthreads();
    const double2 d = D[(size_t)i * NB * NB + q * NB + r], tq = t[q];  // conj(D[q][r]) t_q
    double2 p = make_double2(d.x * tq.x + d.y * tq.y, d.x * tq.y - d.y * tq.x);
    p = chol_sum16(p);
    if (q == 0) y[i * NB + r] = p;
    __syncthreads();
  }
  for (int i = tid; i < P; i += blockDim.x) Rinv[(size_t)i * P + c] = make_float2((float)y[i].x, (float)y[i].y);
}

// The same factorisation and inverse with both triangles resident in LDS
// (P <= kCholLdsMaxP), one workgroup per item: identical arithmetic in the
// same order, so the results are the same bits; the global-memory version
// above serves larger arrays.  Per column: every thread reads the pivot and
// scales its rows of the column, one barrier, the trailing update (and the
// pivot's own store), one barrier.
__global__ __launch_bounds__(256) void chol_inverse_lds_kernel(CholItem one, const CholItem* __restrict__ many,
                                                               int P) {
  __shared__ double2 W[kCholLdsMaxP * (kCholLdsMaxP + 1)];
  __shared__ double2 Li[kCholLdsMaxP * (kCholLdsMaxP + 1)];
  __shared__ int bad;
  const CholItem it = many ? many[blockIdx.x] : one;
  const int tid = threadIdx.x, nt = blockDim.x, LD = P + 1;  // padded rows: column walks spread over the banks
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int e = tid; e < P * P; e += nt) {
    const float2 v = it.R[e];
    if (!isfinite(v.x) || !isfinite(v.y)) bad = 2;
    W[(e / P) * LD + e % P] = make_double2((double)v.x, (double)v.y);
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) *it.status = bad;
    return;
  }
  for (int j = 0; j < P; ++j) {
    const double d = W[j * LD + j].x;  // same value in every thread: the exit below is uniform
    if (!(d > 0.0)) {
      if (tid == 0) *it.status = 1;
      return;
    }
    const double ljj = sqrt(d);
    for (int i = j + 1 + tid; i < P; i += nt) {
      const double2 v = W[i * LD + j];
      W[i * LD + j] = make_double2(v.x / ljj, v.y / ljj);
    }
    __syncthreads();
    if (tid == 0) W[j * LD + j] = make_double2(ljj, 0.0);  // nobody reads the pivot in this phase
    const int m = P - j - 1;
    for (int e = tid; e < m * m; e += nt) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k <= i) {
        const double2 a = W[i * LD + j], b = W[k * LD + j];
        double2 w = W[i * LD + k];
        w.x -= a.x * b.x + a.y * b.y;
        w.y -= a.y * b.x - a.x * b.y;
        W[i * LD + k] = w;
      }
    }
    __syncthreads();
  }
  // Li = L^-1 by forward substitution, one column per thread
  for (int c = tid; c < P; c += nt) {
    for (int i = 0; i < c; ++i) Li[i * LD + c] = make_double2(0.0, 0.0);
    Li[c * LD + c] = make_double2(1.0 / W[c * LD + c].x, 0.0);
    for (int i = c + 1; i < P; ++i) {
      double sr = 0.0, si = 0.0;
      for (int k = c; k < i; ++k) {
        const double2 l = W[i * LD + k], y = Li[k * LD + c];
        sr += l.x * y.x - l.y * y.y;
        si += l.x * y.y + l.y * y.x;
      }
      const double lii = W[i * LD + i].x;
      Li[i * LD + c] = make_double2(-sr / lii, -si / lii);
    }
  }
  __syncthreads();
  for (int e = tid; e < P * P; e += nt) {
    const int i = e / P, k = e % P;
    double sr = 0.0, si = 0.0;
    for (int m = (i > k ? i : k); m < P; ++m) {
      const double2 a = Li[m * LD + i], b = Li[m * LD + k];
      sr += a.x * b.x + a.y * b.y;
      si += a.x * b.y - a.y * b.x;
    }
    it.Rinv[e] = make_float2((float)sr, (float)si);
    if (it.Li) it.Li[e] = Li[i * LD + k];
  }
  if (tid == 0) *it.status = 0;
}

// ---------------------------------------------------------------------------
// Separable steering tables, FP64 phases rounded once to complex64:
//   El[p][il] = P^-1/2 exp(-j 2pi x_p l_il / lambda),  Em[p][im] = exp(-j 2pi y_p m_im / lambda),
// zero rows for the padding antennas p >= P.
// Entry t of the tables of one geometry: the El entries (Pp x nl) first, then
// the Em entries (Pp x nm).
__device__ inline void table_entry(int t, const double* __restrict__ pos, int P, int Pp, double lambda, int nl,
                                   int nm, double l0, double dl, double m0, double dm, float2* __restrict__ El,
                                   float2* __restrict__ Em) {
  const double two_pi = 6.283185307179586476925286766559;
  const double norm = 1.0 / sqrt((double)P);
  const int nEl = Pp * nl;
  const bool is_l = t < nEl;
  const int e = is_l ? t : t - nEl;
  const int n = is_l ? nl : nm;
  const int p = e / n, i = e - p * n;
  float2 v = make_float2(0.f, 0.f);
  if (p < P) {
    const double dir = is_l ? l0 + i * dl : m0 + i * dm;
    const double coord = pos[2 * p + (is_l ? 0 : 1)];
    double sn, cs;
    sincos(-two_pi * coord * dir / lambda, &sn, &cs);
    const double sc = is_l ? norm : 1.0;
    v = make_float2((float)(sc * cs), (float)(sc * sn));
  }
  if (is_l) El[e] = v;
  else Em[e] = v;
}

__global__ void tables_kernel(const double* __restrict__ pos, int P, int Pp, double lambda, int nl,
                              int nm, double l0, double dl, double m0, double dm,
                              float2* __restrict__ El, float2* __restrict__ Em) {
  const int total = Pp * (nl + nm);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x)
    table_entry(t, pos, P, Pp, lambda, nl, nm, l0, dl, m0, dm, El, Em);
}

// per blocks per request
__global__ void tables_batch_kernel(const TableItem* __restrict__ items, int per) {
  const int r = blockIdx.x / per, b = blockIdx.x - r * per;
  const TableItem it = items[r];
  const int Pp = pad_p(it.P), total = Pp * (it.nl + it.nm);
  for (int t = b * blockDim.x + threadIdx.x; t < total; t += per * blockDim.x)
    table_entry(t, it.pos, it.P, Pp, it.lambda, it.nl, it.nm, it.l0, it.dl, it.m0, it.dm, it.El, it.Em);
}

// ---------------------------------------------------------------------------
// Small elementwise helpers.
__global__ void sub_diag_kernel(const float2* __restrict__ R, const float* __restrict__ noise, int P,
                                float2* __restrict__ B0) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < P * P; e += gridDim.x * blockDim.x) {
    float2 v = R[e];
    const int p = e / P, q = e - p * P;
    if (noise && p == q) v.x -= noise[p];
    B0[e] = v;
  }
}

__global__ void fill_kernel(float* __restrict__ x, float v, int n) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) x[e] = v;
}

// ---------------------------------------------------------------------------
// Host-side launchers.
namespace {

template <class Epi>
hipError_t launch_adjoint_epi(const AdjParams& pr, const Epi& epi, hipStream_t st) {
  if (pr.n <= 0) return hipSuccess;
  int T;
  auto go = [&](auto kern, int T_) {
    const int ntiles = (pr.n + T_ - 1) / T_;
    const int grid = ntiles < 4096 ? ntiles : 4096;
    hipLaunchKernelGGL(kern, dim3(grid, pr.blk_grid ? pr.nblk : 1), dim3(kThreads), 0, st, pr, epi);
    return hipGetLastError();
  };
  if (!pr.n_dev) {
    if (pr.MT <= 3) return go(adjoint_kernel<3, 1, 1, Epi>, T = 64);
    if (pr.MT <= 6) return go(adjoint_kernel<6, 1, 1, Epi>, T = 64);
    if (pr.MT <= 12) return go(adjoint_kernel<12, 1, 1, Epi>, T = 64);
  }
  const int ngroups = (pr.MT + 3) / 4;
  // a list built on the device (usually short): one tile per workgroup, at
  // most 16 workgroups along the list (striding over longer lists), the most
  // K slices
  const int nt = pr.n_dev ? 1 : (pr.n <= 16 ? 1 : (pr.n <= 32 ? 2 : 4));
  const int xt0 = (pr.n + 16 * nt - 1) / (16 * nt);
  const int xt = pr.n_dev ? std::min(xt0, 16) : xt0;
  // K slices: about 256 workgroups in all, at least 16 chunks per slice
  int ksl = pr.n_dev ? 8 : (256 + xt * ngroups - 1) / (xt * ngroups);
  ksl = std::max(1, std::min(ksl, std::min(8, pr.KS / 16)));
  if (pr.rows_part && pr.frag && !pr.U && !pr.xf && pr.nblk == 1 &&
      (size_t)ngroups * ksl * pr.n <= pr.rows_cap) {
    // rows and K split over workgroups, then the ordered sum and the epilogue
    // on the same pixel tiles as adjoint_kernel
    const int T_ = adjoint_tile_width(pr.MT);
    const dim3 g1(xt, ngroups, ksl);
    if (nt == 1) hipLaunchKernelGGL(adjoint_rows_kernel<1>, g1, dim3(kThreads), 0, st, pr, pr.rows_part);
    else if (nt == 2) hipLaunchKernelGGL(adjoint_rows_kernel<2>, g1, dim3(kThreads), 0, st, pr, pr.rows_part);
    else hipLaunchKernelGGL(adjoint_rows_kernel<4>, g1, dim3(kThreads), 0, st, pr, pr.rows_part);
    hipLaunchKernelGGL(adjoint_rows_finish_kernel<Epi>, dim3((pr.n + T_ - 1) / T_), dim3(64), 0, st, pr,
                       (const float*)pr.rows_part, ngroups * ksl, T_, epi);
    return hipGetLastError();
  }
  if (pr.n_dev) return hipErrorInvalidValue;  // a device-length list needs the row-split kernel
  if (pr.MT <= 24) return go(adjoint_kernel<6, 2, 4, Epi>, T = 32);
  return go(adjoint_kernel<9, 4, 4, Epi>, T = 64);
}

}  // namespace

int adjoint_tile_width(int MT) { return (MT > 12 && MT <= 24) ? 32 : 64; }

// Narrow tiles (two waves split the rows, T = 32) for the small free sets of
// the LSQR subproblems when the row tiles divide evenly.
// For 7..12 row tiles the four waves split the rows (three tiles each) over
// 16-pixel tiles, so that even small free sets spread over several CUs.
int adjoint_lsqr2_tile_width(int MT, int n) {
  if (MT > 6 && MT <= 12) return 16;
  return (MT <= 6 && n <= 1024) ? 32 : adjoint_tile_width(MT);
}

hipError_t launch_adjoint_lsqr2(const AdjParams& pr, const EpiLsqrV2& epi, hipStream_t st) {
  if (pr.n <= 0) return hipSuccess;
  if (pr.MT > 6 && pr.MT <= 12) {
    const dim3 g((pr.n + 15) / 16), b(kThreads);
    if (pr.xf && pr.frag && !pr.U) {
      const dim3 bl(64 * pr.MT);  // one wave per row tile
      switch (pr.MT) {
        case 7: hipLaunchKernelGGL((adjoint_list_kernel<7>), g, bl, 0, st, pr, epi); break;
        case 8: hipLaunchKernelGGL((adjoint_list_kernel<8>), g, bl, 0, st, pr, epi); break;
        case 9: hipLaunchKernelGGL((adjoint_list_kernel<9>), g, bl, 0, st, pr, epi); break;
        case 10: hipLaunchKernelGGL((adjoint_list_kernel<10>), g, bl, 0, st, pr, epi); break;
        case 11: hipLaunchKernelGGL((adjoint_list_kernel<11>), g, bl, 0, st, pr, epi); break;
        default: hipLaunchKernelGGL((adjoint_list_kernel<12>), g, bl, 0, st, pr, epi); break;
      }
    } else {
      hipLaunchKernelGGL((adjoint_kernel<3, 1, 4, EpiLsqrV2>), g, b, 0, st, pr, epi);
    }
    return hipGetLastError();
  }
  if (adjoint_lsqr2_tile_width(pr.MT, pr.n) == 32 && pr.MT <= 6) {
    const int ntiles = (pr.n + 31) / 32;
    if (pr.MT <= 3)
      hipLaunchKernelGGL((adjoint_kernel<2, 1, 2, EpiLsqrV2>), dim3(ntiles), dim3(kThreads), 0, st, pr, epi);
    else
      hipLaunchKernelGGL((adjoint_kernel<3, 1, 2, EpiLsqrV2>), dim3(ntiles), dim3(kThreads), 0, st, pr, epi);
    return hipGetLastError();
  }
  return launch_adjoint_epi(pr, epi, st);
}

hipError_t launch_adjoint_store(const AdjParams& pr, float* out, float scale, hipStream_t st) {
  return launch_adjoint_epi(pr, EpiStore{out, scale}, st);
}
hipError_t launch_adjoint_mf(const AdjParams& pr, float* mf, float* eps, float eps_scale,
                             hipStream_t st) {
  return launch_adjoint_epi(pr, EpiMF{mf, eps, eps_scale}, st);
}
hipError_t launch_adjoint_mvdr(const AdjParams& pr, float* gamma, double C, double kb_coef,
                               hipStream_t st) {
  return launch_adjoint_epi(pr, EpiMVDR{gamma, C, kb_coef}, st);
}
hipError_t launch_adjoint_lambda(const AdjParams& pr, const uint8_t* state, uint64_t* part,
                                 hipStream_t st) {
  return launch_adjoint_epi(pr, EpiLambda{state, part}, st);
}
hipError_t launch_adjoint_lsqr(const AdjParams& pr, float* v, const double* beta_part, int nbeta,
                               double* alpha_part, int init, hipStream_t st) {
  return launch_adjoint_epi(pr, EpiLsqrV{v, beta_part, nbeta, alpha_part, init}, st);
}
// both adjoint paths put the epilogue of tiles of adjoint_tile_width(MT)
// pixels in one workgroup each
bool adjoint_lsqr_fuses(const AdjParams& pr) {
  return !pr.n_dev && !pr.blk_grid && pr.nblk == 1 && pr.n >= 1 && pr.n <= adjoint_tile_width(pr.MT);
}
hipError_t launch_adjoint_lsqr_step(const AdjParams& pr, float* v, const double* beta_part, int nbeta,
                                    double* alpha_part, LsqrState* ls, float* w, float* x, hipStream_t st) {
  if (!adjoint_lsqr_fuses(pr)) return hipErrorInvalidValue;
  EpiLsqrV e{v, beta_part, nbeta, alpha_part, 0};
  e.ls = ls;
  e.w = w;
  e.x = x;
  return launch_adjoint_epi(pr, e, st);
}
hipError_t launch_adjoint_store_blocks(const AdjParams& pr, float* out, size_t stride, hipStream_t st) {
  AdjParams p = pr;
  p.blk_grid = 1;
  return launch_adjoint_epi(p, EpiStoreBlk{out, stride}, st);
}

// Partials of the correlation: at most this many chunks (workgroups along
// the list) per block pair.
int forward_chunks_max(int P) {
  return std::max(1, 2048 / corr_pairs(P));
}
size_t forward_part_floats(int P) { return (size_t)corr_pairs(P) * corr_bt(P) * corr_bt(P) * 512; }

// Up to about 2048 workgroups over all block pairs, at least 256 pixels
// (16 k steps per wave) per workgroup unless the list is shorter: fewer,
// longer chunks keep the partials (and the reduction's serial sums) small.
void forward_plan(int P, int n, int* chw, int* nchunks) {
  const int maxc = forward_chunks_max(P);
  int c = (n + maxc - 1) / maxc;
  c = std::max(std::min(256, (n + 15) & ~15), (c + 15) & ~15);
  c = std::max(16, c);
  *chw = c;
  *nchunks = n > 0 ? (n + c - 1) / c : 0;
}

hipError_t launch_forward(const FwdParams& pr, hipStream_t st) {
  if (pr.n <= 0) return hipSuccess;
  const int P = pr.tab.Pp;  // corr_* depend on Pp only
  const int nchunks = (pr.n + pr.chw - 1) / pr.chw;
  const dim3 grid(nchunks, corr_pairs(P), pr.nblk);
  const bool tr = pr.tab.ElT && pr.tab.EmT && pr.nblk == 1, list = pr.idx != nullptr;
#define CORR_LAUNCH(BT_, TR_, LIST_) hipLaunchKernelGGL((corr_kernel<BT_, TR_, LIST_>), grid, dim3(kThreads), 0, st, pr)
#define CORR_LIST(BT_, TR_)   \
  if (list) {                 \
    CORR_LAUNCH(BT_, TR_, true);  \
  } else {                    \
    CORR_LAUNCH(BT_, TR_, false); \
  }
  if (corr_bt(P) == 2) {
    if (tr) {
      CORR_LIST(2, true)
    } else {
      CORR_LIST(2, false)
    }
  } else {
    if (tr) {
      CORR_LIST(3, true)
    } else {
      CORR_LIST(3, false)
    }
  }
#undef CORR_LIST
#undef CORR_LAUNCH
  return hipGetLastError();
}

int reduce_blocks(int P) {
  const int na = corr_tiles(P);
  return na * (na + 1) / 2;  // one workgroup (and one norm partial) per antenna tile pair
}

hipError_t launch_reduce(const RedParams& pr, hipStream_t st) {
  hipLaunchKernelGGL(reduce_kernel, dim3(reduce_blocks(pr.P), pr.nblk), dim3(256 * kRedGroups), 0, st, pr);
  return hipGetLastError();
}

bool corr_small_fits(int n, int nblk) { return n >= 1 && n <= kCorrSmall && nblk == 1; }

hipError_t launch_corr_small(const FwdParams& f, const RedParams& pr, hipStream_t st) {
  if (!corr_small_fits(f.n, pr.nblk) || f.nblk != 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(corr_small_kernel, dim3(reduce_blocks(pr.P)), dim3(256), 0, st, f, pr);
  return hipGetLastError();
}

size_t chol_work_elems(int P) {
  const size_t nbk = (size_t)(P + kCholNB - 1) / kCholNB;
  return (size_t)2 * P * P + nbk * kCholNB * kCholNB;
}

hipError_t launch_chol_inverse(const float2* R, int P, double2* W, double2* Li, float2* Rinv,
                               int* status, hipStream_t st) {
  if (P <= kCholLdsMaxP) {
    const CholItem one{R, Li, Rinv, status};
    hipLaunchKernelGGL(chol_inverse_lds_kernel, dim3(1), dim3(256), 0, st, one, (const CholItem*)nullptr, P);
  } else {
    if (P > kCholMaxRows) return hipErrorInvalidValue;
    // W holds two P x P FP64 matrices, L (row-major) and its transpose, then the inverses of the
    // diagonal blocks (chol_work_elems)
    double2* LT = W + (size_t)P * P;
    double2* D = LT + (size_t)P * P;
    const int nbk = (P + kCholNB - 1) / kCholNB;
    hipLaunchKernelGGL(chol_convert_kernel, dim3(1), dim3(1024), 0, st, R, P, W, LT, D, status);
    for (int j0 = 0; j0 + kCholNB < P; j0 += kCholNB) {
      const int T = (P - j0 - kCholNB + kCholTile - 1) / kCholTile;
      hipLaunchKernelGGL(chol_update_kernel, dim3(T * (T + 1) / 2), dim3(256), 0, st, W, LT, D, P, j0, status);
    }
    hipLaunchKernelGGL(chol_lower_kernel, dim3(nbk - 1), dim3(256), 0, st, W, (const double2*)LT, P,
                       (const int*)status);
    hipLaunchKernelGGL(chol_solve_kernel, dim3(P), dim3(256), 0, st, (const double2*)W, (const double2*)LT,
                       (const double2*)D, P, (const int*)status, Li, Rinv);
  }
  return hipGetLastError();
}

hipError_t launch_chol_inverse_batch(const CholItem* items, int n, int P, hipStream_t st) {
  if (P > kCholLdsMaxP || n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(chol_inverse_lds_kernel, dim3(n), dim3(256), 0, st, CholItem{}, items, P);
  return hipGetLastError();
}

hipError_t launch_tables_batch(const TableItem* items, int nreq, int total_max, hipStream_t st) {
  const int per = std::max(1, std::min(16, (total_max + kThreads - 1) / kThreads));
  hipLaunchKernelGGL(tables_batch_kernel, dim3(nreq * per), dim3(kThreads), 0, st, items, per);
  return hipGetLastError();
}

// Antenna-fastest copies of the steering tables: T[i][p] = E[p][i] for
// p < Pp, zero up to the row length corr_rows(Pp).
__global__ __launch_bounds__(kThreads) void tables_t_kernel(const float2* __restrict__ El, const float2* __restrict__ Em,
                                                          int Pp, int nl, int nm, float2* __restrict__ ElT,
                                                          float2* __restrict__ EmT) {
  const int rowT = corr_rows(Pp);
  const int nt = rowT * (nl + nm);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nt; e += gridDim.x * blockDim.x) {
    const int p = e % rowT, r = e / rowT;  // consecutive threads: consecutive antennas of one pixel row
    if (r < nl) ElT[e] = p < Pp ? El[(size_t)p * nl + r] : make_float2(0.f, 0.f);
    else EmT[(size_t)(r - nl) * rowT + p] = p < Pp ? Em[(size_t)p * nm + (r - nl)] : make_float2(0.f, 0.f);
  }
}

hipError_t launch_tables_t(const float2* El, const float2* Em, int Pp, int nl, int nm, float2* ElT, float2* EmT,
                           hipStream_t st) {
  int grid = (corr_rows(Pp) * (nl + nm) + kThreads - 1) / kThreads;
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(tables_t_kernel, dim3(grid), dim3(kThreads), 0, st, El, Em, Pp, nl, nm, ElT, EmT);
  return hipGetLastError();
}

hipError_t launch_tables(const double* pos, int P, double lambda, int nl, int nm, double l0,
                         double dl, double m0, double dm, float2* El, float2* Em, hipStream_t st) {
  const int Pp = pad_p(P);
  const int total = Pp * (nl + nm);
  int grid = (total + kThreads - 1) / kThreads;
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(tables_kernel, dim3(grid), dim3(kThreads), 0, st, pos, P, Pp, lambda, nl, nm,
                     l0, dl, m0, dm, El, Em);
  return hipGetLastError();
}

hipError_t launch_sub_diag(const float2* R, const float* noise, int P, float2* B0, hipStream_t st) {
  const int grid = (P * P + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(sub_diag_kernel, dim3(grid), dim3(kThreads), 0, st, R, noise, P, B0);
  return hipGetLastError();
}

hipError_t launch_fill(float* x, float v, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int grid = (n + kThreads - 1) / kThreads;
  if (grid > 2048) grid = 2048;
  hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(kThreads), 0, st, x, v, n);
  return hipGetLastError();
}

}  // namespace clsimg
