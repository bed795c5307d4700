// Register-resident beamformer g_i = Re(a_i^H U a_i) over a whole pixel grid
// (the adjoint of Sec. IV-C, eq. psiH, on all pixels: the dirty image of
// eq. mfdimg, the MVDR power of eq. wmvdr and the gradient of eq. gls).
//
// With x_i the real embedding of a_i, g_i = x_i^T Ut x_i.  The embedding is
// ordered so that one MFMA lane generates whole complex entries: position
// 4 kc + q (kc = 0 .. 2Pp/4 - 1, q = 0 .. 3) holds component (kc & 1) of
// antenna 4 (kc >> 1) + q.  In that order Ut is split into 16 x 16 tiles and
// only the lower block triangle is kept, off-diagonal tiles doubled:
//   x^T Ut x = sum_m x_m^T Ut_mm x_m + 2 sum_{k<m} x_m^T Ut_mk x_k.
// Inside each row tile the rows are stored transposed in (q, r) (row
// 16m + 4q + r holds tile row 16m + 4r + q), so that after the MFMAs the
// accumulator element r of lane (c16, q) multiplies exactly the B operand
// that lane loaded for chunk kc = 4m + r: the column dot needs no exchange
// between lanes beyond the final sum over q.
//
// Each wave holds all 2 MT (MT + 1) fragment registers of Ut for the whole
// launch (built once per workgroup from U through LDS, or loaded prepared) and
// walks 16-pixel tiles; it generates the steering entries of its tile from the
// separable tables (one complex product per entry).  After the fragments are
// in registers there is no LDS traffic and no barrier on the path.
#include <utility>

#include "kernels.h"

namespace clsimg {

constexpr int kBeamWaves = 4;
constexpr int kBeamMaxMT = 6;

// embedding position -> (antenna, component)
__device__ __forceinline__ void beam_pos(int idx, int& p, int& s) {
  const int kc = idx >> 2, q = idx & 3;
  p = 4 * (kc >> 1) + q;
  s = kc & 1;
}

// Fragment f = 2 m (m + 1) + kc (kc < 4 (m + 1)) for lane l holds
// Ut[rowpos][4 kc + (l >> 4)] with rowpos = 16 m + 4 ((l & 15) & 3) + ((l & 15) >> 2),
// Ut built from the Hermitian part of U (which leaves Re(a^H U a) unchanged).
__global__ void beam_prep_kernel(const float2* __restrict__ U, int P, int MT, float* __restrict__ frag) {
  const int nfr = 2 * MT * (MT + 1);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nfr * 64; e += gridDim.x * blockDim.x) {
    const int f = e >> 6, l = e & 63;
    int m = 0;
    while (2 * (m + 1) * (m + 2) <= f) ++m;
    const int kc = f - 2 * m * (m + 1);
    const int c16 = l & 15, qq = l >> 4;
    int p, s, p2, t;
    beam_pos(16 * m + 4 * (c16 & 3) + (c16 >> 2), p, s);
    beam_pos(4 * kc + qq, p2, t);
    float v = 0.f;
    if (p < P && p2 < P) {
      const float2 x = U[p * P + p2], y = U[p2 * P + p];
      const float hr = 0.5f * (x.x + y.x), hi = 0.5f * (x.y - y.y);
      v = (s == t) ? hr : (s == 0 ? -hi : hi);
      if ((kc >> 2) < m) v *= 2.f;
    }
    frag[e] = v;
  }
}

struct BeamMF {
  float* mf;
  float* eps;
  float eps_scale;
  __device__ void init() {}
  __device__ void operator()(int pix, float g, bool ok) {
    if (ok) {
      mf[pix] = g;
      if (eps) eps[pix] = g * eps_scale;
    }
  }
  __device__ void finish(int) {}
};

struct BeamMVDR {
  float* gamma;
  double C, kb_coef;
  __device__ void init() {}
  __device__ void operator()(int pix, float g, bool ok) {
    if (ok) {
      const double h = (double)g;
      gamma[pix] = (float)(C / h + kb_coef / h);
    }
  }
  __device__ void finish(int) {}
};

struct BeamStore {
  float* out;
  float scale;
  __device__ void init() {}
  __device__ void operator()(int pix, float g, bool ok) {
    if (ok) out[pix] = g * scale;
  }
  __device__ void finish(int) {}
};

// Sums over covariance blocks: sum[i] (+)= scale * g_i and, if sumsq is
// given, sumsq[i] (+)= g_i^2 (first block: =).  The blocks are added in order.
struct BeamAcc {
  float* sum;
  float* sumsq;
  float scale;
  int first;
  __device__ void init() {}
  __device__ void operator()(int pix, float g, bool ok) {
    if (ok) {
      const float v = g * scale;
      sum[pix] = first ? v : sum[pix] + v;
      if (sumsq) sumsq[pix] = first ? g * g : sumsq[pix] + g * g;
    }
  }
  __device__ void finish(int) {}
};

// Lagrange multipliers of the active pixels (eqs. etaL, etaU): lambda = g on
// L, -g on U; the block's smallest key (ordered lambda << 32 | pixel, so ties
// go to the lowest pixel) is written to part[blockIdx.x].
struct BeamLambda {
  const uint8_t* state;
  uint64_t* part;
  const float* scale;  // optional positive per-pixel factor (PWLS: 1 / D_i)
  uint64_t best;
  __device__ void init() { best = ~0ull; }
  __device__ void operator()(int pix, float g, bool ok) {
    if (ok) {
      const uint8_t s = state[pix];
      if (s != 1) {  // not free
        if (scale) g *= scale[pix];
        const float lam = (s == 0) ? g : -g;  // L : U
        const uint64_t key = ((uint64_t)ordered_bits(lam) << 32) | (uint32_t)pix;
        best = key < best ? key : best;
      }
    }
  }
  // The register beamformer loads the state (and scale) of a tile's pixel
  // together with the tile's table entries, one tile ahead, so the epilogue
  // does not wait for them: prefetch(pix) for the next tile, begin_tile()
  // when it becomes current, then apply() in place of operator().
  uint8_t s_next, s_cur;
  float sc_next, sc_cur;
  __device__ void prefetch(int pix) {
    s_next = ld_global(state + pix);
    sc_next = scale ? ld_global(scale + pix) : 1.f;
  }
  __device__ void begin_tile() {
    s_cur = s_next;
    sc_cur = sc_next;
  }
  __device__ void apply(int pix, float g, bool ok) {
    if (ok && s_cur != 1) {  // not free
      if (scale) g *= sc_cur;
      const float lam = (s_cur == 0) ? g : -g;  // L : U
      const uint64_t key = ((uint64_t)ordered_bits(lam) << 32) | (uint32_t)pix;
      best = key < best ? key : best;
    }
  }
  __device__ void finish(int blk) {
    __shared__ uint64_t sh[kBeamWaves];
    const uint64_t m = block_min_u64(best, sh);
    if (threadIdx.x == 0) part[blk] = m;
  }
};

// Epilogues with per-pixel inputs load them one tile ahead (prefetch /
// begin_tile / apply); the others take the value at once.
template <class E>
__device__ __forceinline__ auto epi_prefetch(E& e, int pix, int) -> decltype(e.prefetch(pix), void()) {
  e.prefetch(pix);
}
template <class E>
__device__ __forceinline__ void epi_prefetch(E&, int, long) {}
template <class E>
__device__ __forceinline__ auto epi_begin(E& e, int) -> decltype(e.begin_tile(), void()) {
  e.begin_tile();
}
template <class E>
__device__ __forceinline__ void epi_begin(E&, long) {}
template <class E>
__device__ __forceinline__ auto epi_apply(E& e, int pix, float g, bool ok, int) -> decltype(e.apply(pix, g, ok), void()) {
  e.apply(pix, g, ok);
}
template <class E>
__device__ __forceinline__ void epi_apply(E& e, int pix, float g, bool ok, long) {
  e(pix, g, ok);
}

// Fragments built from U by the whole workgroup: the (m, j) pairs of chunks
// 2j, 2j + 1 of row tile m (same values as beam_prep_kernel) are dealt round
// robin to the waves, written to LDS and then read back by every wave.  For
// row tile m the lane's row is antenna 8m + 4((c16 >> 1) & 1) + (c16 >> 2),
// component c16 & 1; the pair shares column antenna 4j + q and takes the two
// components of the same Hermitian-part entry.  In LDS fragment f of lane l
// sits at (f >> 2) * 256 + 4 l + (f & 3): a pair is one 8-byte store and each
// lane reads its fragments four at a time with 16-byte loads.
template <int MT, class Issue>
__device__ __forceinline__ void beam_frags_from_u(const float2* __restrict__ U, int P, float* sfr, float* fa,
                                                  Issue&& issue_next) {
  constexpr int NPAIR = MT * (MT + 1);
  constexpr int NFR = 2 * NPAIR;
  constexpr int PPW = (NPAIR + kBeamWaves - 1) / kBeamWaves;
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int pr0 = 4 * ((c16 >> 1) & 1) + (c16 >> 2);
  const bool s1 = c16 & 1;
  float2 xv[PPW], yv[PPW];
  int mm[PPW], jj[PPW];
#pragma unroll
  for (int i = 0; i < PPW; ++i) {
    const int t = min(w + kBeamWaves * i, NPAIR - 1);
    int m = 0;
    while ((m + 1) * (m + 2) <= t) ++m;
    mm[i] = m;
    jj[i] = t - m * (m + 1);
    // clamped (valid) indices, padding masked afterwards: no branch around a
    // load, so all of them are in flight together
    const int p = min(8 * m + pr0, P - 1), p2 = min(4 * jj[i] + q, P - 1);
    xv[i] = ld_global(U + p * P + p2);
    yv[i] = ld_global(U + p2 * P + p);
  }
  // the caller's next loads go out behind these (loads complete in order, so
  // waiting for the U entries does not wait for them)
  issue_next();
#pragma unroll
  for (int i = 0; i < PPW; ++i) {
    if (w + kBeamWaves * i < NPAIR) {
      const int m = mm[i], j = jj[i];
      const bool live = 8 * m + pr0 < P && 4 * j + q < P;
      const float d = (j >> 1) < m ? 2.f : 1.f;  // chunks 2j, 2j+1 lie in column tile j >> 1
      const float hr = live ? 0.5f * d * (xv[i].x + yv[i].x) : 0.f;
      const float hi = live ? 0.5f * d * (xv[i].y - yv[i].y) : 0.f;
      const int f = 2 * m * (m + 1) + 2 * j;  // even
      *reinterpret_cast<float2*>(sfr + (f >> 2) * 256 + 4 * lane + (f & 3)) =
          make_float2(s1 ? hi : hr, s1 ? hr : -hi);
    }
  }
  __syncthreads();
  static_assert(NFR % 4 == 0, "fragments are read four at a time");
#pragma unroll
  for (int f4 = 0; f4 < NFR / 4; ++f4) {
    const float4 v = *reinterpret_cast<const float4*>(sfr + f4 * 256 + 4 * lane);
    fa[4 * f4] = v.x;
    fa[4 * f4 + 1] = v.y;
    fa[4 * f4 + 2] = v.z;
    fa[4 * f4 + 3] = v.w;
  }
}

template <int MT, class Epi>
__device__ __forceinline__ void beam_body(const float* __restrict__ frag, const float2* __restrict__ U, int P,
                                          const Tables& tab, const int* skip, Epi& epi, int blk, int nblk) {
  constexpr int KS = 4 * MT;             // 4-row chunks of the embedding
  constexpr int NFR = 2 * MT * (MT + 1);  // fragments of the lower block triangle
  if (skip && ld_global(skip)) return;
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
  const int Q = tab.Q, nl = tab.nl, nm = tab.nm;
  const int ntiles = (Q + 15) >> 4;
  const int nwav = nblk * kBeamWaves;
  // table entries of antennas 4 j + q for this lane's pixel of a tile; the
  // loads of the next tile are issued before the current one is multiplied.
  // The first tile's loads go out right behind the loads of U, so their
  // latency overlaps the fragment build.
  float2 te[KS / 2], tm[KS / 2];
  auto load_tables = [&](int tile) {
    const int pix = min(16 * tile + c16, Q - 1);
    const int im = pix / nl, il = pix - im * nl;
    const float2* el = tab.El + (size_t)q * nl + il;
    const float2* em = tab.Em + (size_t)q * nm + im;
#pragma unroll
    for (int j = 0; j < KS / 2; ++j) {
      te[j] = ld_global(el + (size_t)4 * j * nl);
      tm[j] = ld_global(em + (size_t)4 * j * nm);
    }
  };
  // workgroups are dealt round robin to the 8 XCDs: give each XCD a
  // contiguous run of tiles (whole image rows), so that its L2 holds only its
  // rows' part of the m table rather than every XCD fetching all of it
  if (nblk % 8 == 0) blk = (blk % 8) * (nblk / 8) + blk / 8;
  int tile = blk * kBeamWaves + (threadIdx.x >> 6);
  auto first_loads = [&]() {
    if (tile < ntiles) {
      load_tables(tile);
      epi_prefetch(epi, min(16 * tile + c16, Q - 1), 0);
    }
  };
  float fa[NFR];
  if (U) {
    __shared__ __align__(16) float sfr[NFR * 64];
    beam_frags_from_u<MT>(U, P, sfr, fa, first_loads);
  } else {
#pragma unroll
    for (int f = 0; f < NFR; ++f) fa[f] = frag[f * 64 + lane];
    first_loads();
  }
  epi.init();
  for (; tile < ntiles; tile += nwav) {
    const int pix = 16 * tile + c16;
    epi_begin(epi, 0);
    float b[KS];
#pragma unroll
    for (int j = 0; j < KS / 2; ++j) {
      const float2 a = cmul(te[j], tm[j]);
      b[2 * j] = a.x;
      b[2 * j + 1] = a.y;
    }
    if (tile + nwav < ntiles) {
      load_tables(tile + nwav);
      epi_prefetch(epi, min(16 * (tile + nwav) + c16, Q - 1), 0);
    }
    v4f acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KS; ++kc) {
#pragma unroll
      for (int m = kc >> 2; m < MT; ++m) acc[m] = mfma16x16x4(fa[2 * m * (m + 1) + kc], b[kc], acc[m]);
    }
    float g = 0.f;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
#pragma unroll
      for (int r = 0; r < 4; ++r) g += acc[m][r] * b[4 * m + r];
    }
    g += __shfl_xor(g, 16, 64);
    g += __shfl_xor(g, 32, 64);
    epi_apply(epi, pix, g, pix < Q && q == 0, 0);
  }
  epi.finish(blk);
}

// (at most two waves per SIMD: the fragments, the tile's operands and the
// accumulators all stay in registers)
template <int MT, class Epi>
__global__ __launch_bounds__(64 * kBeamWaves) __attribute__((amdgpu_waves_per_eu(1, 2))) void beam_kernel(
    const float* __restrict__ frag, const float2* __restrict__ U, int P, Tables tab, const int* skip, Epi epi) {
  beam_body<MT>(frag, U, P, tab, skip, epi, blockIdx.x, gridDim.x);
}

// Multipliers of a batch of requests in one launch: bpr blocks per request.
template <int MT>
__global__ __launch_bounds__(64 * kBeamWaves) __attribute__((amdgpu_waves_per_eu(1, 2))) void beam_lambda_batch_kernel(
    const BeamLamItem* __restrict__ items, int bpr) {
  const int r = blockIdx.x / bpr, lb = blockIdx.x - r * bpr;
  const BeamLamItem it = items[r];
  if (lb >= it.nblk) return;  // the whole block: this request has fewer pixels
  BeamLambda epi{it.state, it.part, it.scale, 0};
  beam_body<MT>(nullptr, it.U, it.P, it.tab, it.skip, epi, lb, it.nblk);
}

// Set-up beamformers of a batch of requests: grid.x runs over nreq x bpr
// blocks, grid.y picks the dirty image (0) or the MVDR bound (1).
template <int MT>
__global__ __launch_bounds__(64 * kBeamWaves) __attribute__((amdgpu_waves_per_eu(1, 2))) void beam_setup_batch_kernel(
    const BeamSetItem* __restrict__ items, int bpr) {
  const int r = blockIdx.x / bpr, lb = blockIdx.x - r * bpr;
  const BeamSetItem it = items[r];
  if (lb >= it.nblk) return;
  if (blockIdx.y == 0) {
    BeamMF epi{it.mf, it.eps, it.eps_scale};
    beam_body<MT>(nullptr, it.R, it.P, it.tab, nullptr, epi, lb, it.nblk);
  } else {
    BeamMVDR epi{it.gamma, it.C, it.kb};
    beam_body<MT>(nullptr, it.Rinv, it.P, it.tab, nullptr, epi, lb, it.nblk);
  }
}

// ---------------------------------------------------------------------------
// Larger arrays (P > 48): the fragments of the whole Ut no longer fit in
// registers, so the product is organised like a GEMM.  A workgroup takes NT
// 16-pixel tiles (two, four or eight); wave w owns RPW row tiles, m = 4i + w
// for even i and 4i + 3 - w for odd i (so that the four waves carry the same
// work), and streams their fragments from L2 while it generates the B
// operands of its pixel tiles from the tables, one complex product per two
// 4-row chunks.  Ut is symmetric, so x^T Ut x = sum_m x_m^T Ut_mm x_m +
// 2 sum_{c<m} x_m^T Ut_mc x_c over 16 x 16 blocks: row tile m runs the chunks
// of column tiles 0..m only, with the fragments of c < m doubled by
// beam_prep_full_kernel (same row permutation as above); that is 51 % of the
// full product's MFMAs at 288 antennas.  After the K loop the column dot needs
// the lane's entries of its own row tiles again: they are recomputed from the
// tables (two complex products per row tile and pixel tile).  The four waves'
// partial sums meet in LDS.
__host__ __device__ inline int big_rpw(int MT) { return (MT + 3) / 4; }
// 16-pixel tiles per workgroup.  The default (measured: two for up to 16 row
// tiles, where more workgroups hide the load latency, four for longer K
// loops, where the fragment loads are shared by more MFMAs) can be replaced
// by an autotuned choice among kBigNT; every choice computes each pixel with
// the same operations in the same order.
__host__ __device__ constexpr int big_nt(int rpw) { return rpw <= 4 ? 2 : 4; }
// eight tiles only up to 6 row tiles per wave: beyond, the accumulators no
// longer fit in the register file
__host__ __device__ constexpr bool big_nt_ok(int nt, int rpw) { return nt == 2 || nt == 4 || (nt == 8 && rpw <= 6); }
__host__ __device__ inline int big_nt_or(int nt, int rpw) { return big_nt_ok(nt, rpw) ? nt : big_nt(rpw); }

__global__ void beam_prep_full_kernel(const float2* __restrict__ U, int P, int MT, float* __restrict__ frag) {
  const int KS = 4 * MT, rows = 4 * big_rpw(MT);
  const int total = rows * KS * 64;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int f = e >> 6, l = e & 63;
    const int m = f / KS, kc = f - m * KS;
    const int c16 = l & 15, qq = l >> 4;
    int p, s, p2, t;
    beam_pos(16 * m + 4 * (c16 & 3) + (c16 >> 2), p, s);
    beam_pos(4 * kc + qq, p2, t);
    float v = 0.f;
    const int ct = kc >> 2;  // column tile: below the diagonal doubled, above it unused (zero)
    if (m < MT && p < P && p2 < P && ct <= m) {
      const float2 x = U[p * P + p2], y = U[p2 * P + p];
      const float hr = 0.5f * (x.x + y.x), hi = 0.5f * (x.y - y.y);
      v = (s == t) ? hr : (s == 0 ? -hi : hi);
      if (ct < m) v *= 2.f;
    }
    frag[e] = v;
  }
}

template <int RPW, int NT, class Epi>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void beam_big_kernel(
    const float* __restrict__ frag, int MT, Tables tab, const int* skip, Epi epi) {
  if (skip && *skip) return;
  __shared__ float gsum[4][NT * 16];
  __shared__ float2 bsh[2][NT][64];  // B operands of a chunk pair, per tile and lane (double buffer)
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
  // wave index as a scalar: the row-tile tests below are wave-uniform branches
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int KS = 4 * MT;
  const int Q = tab.Q, nl = tab.nl, nm = tab.nm;
  const int ntiles = (Q + 15) >> 4;
  int mrow[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) mrow[i] = 4 * i + ((i & 1) ? 3 - w : w);
  // the waves share one barrier per chunk pair, so every wave runs all of them
  const int jend = KS / 2;
  constexpr int GT = (NT + 3) / 4;  // tiles whose operands this wave generates: w, w + 4
  epi.init();
  for (int blk = blockIdx.x; blk * NT < ntiles; blk += gridDim.x) {
    // operand generation: tile w + 4 tt, this lane's pixel, antennas 4j + q
    const float2* elg[GT];
    const float2* emg[GT];
#pragma unroll
    for (int tt = 0; tt < GT; ++tt) {
      const int t = min(w + 4 * tt, NT - 1);
      const int pix = min(16 * (blk * NT + t) + c16, Q - 1);
      const int im = pix / nl, il = pix - im * nl;
      elg[tt] = tab.El + (size_t)q * nl + il;
      emg[tt] = tab.Em + (size_t)q * nm + im;
    }
    float2 te[GT], tm[GT];
    auto issue = [&](int jj) {
#pragma unroll
      for (int tt = 0; tt < GT; ++tt) {
        te[tt] = elg[tt][(size_t)4 * jj * nl];
        tm[tt] = emg[tt][(size_t)4 * jj * nm];
      }
    };
    auto store = [&](int slot) {
#pragma unroll
      for (int tt = 0; tt < GT; ++tt)
        if (w + 4 * tt < NT) bsh[slot][w + 4 * tt][lane] = cmul(te[tt], tm[tt]);
    };
    v4f acc[RPW][NT];
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[i][t] = v4f{0.f, 0.f, 0.f, 0.f};
    float f0n[RPW], f1n[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const float* fr = frag + (size_t)min(mrow[i], MT - 1) * KS * 64 + lane;
      f0n[i] = fr[0];
      f1n[i] = fr[64];
    }
    issue(0);
    store(0);
    if (jend > 1) issue(1);
    __syncthreads();
    for (int j = 0; j < jend; ++j) {  // chunk pair 2j, 2j + 1: antenna 4j + q, column tile j >> 1
      const int ct = j >> 1;
      if (j + 1 < jend) {  // the next pair's operands into the other slot, loads for the one after
        store((j + 1) & 1);
        if (j + 2 < jend) issue(j + 2);
      }
      float f0[RPW], f1[RPW];
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        f0[i] = f0n[i];
        f1[i] = f1n[i];
      }
      const int jn = j + 1 < jend ? j + 1 : j;
      const int ctn = jn >> 1;
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        if (mrow[i] >= ctn && mrow[i] < MT) {  // wave-uniform
          const float* fr = frag + ((size_t)mrow[i] * KS + 2 * jn) * 64 + lane;
          f0n[i] = fr[0];
          f1n[i] = fr[64];
        }
      }
      float b0[NT], b1[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const float2 a = bsh[j & 1][t][lane];
        b0[t] = a.x;
        b1[t] = a.y;
      }
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        if (mrow[i] >= ct && mrow[i] < MT) {  // wave-uniform
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            acc[i][t] = mfma16x16x4(f0[i], b0[t], acc[i][t]);
            acc[i][t] = mfma16x16x4(f1[i], b1[t], acc[i][t]);
          }
        }
      }
      __syncthreads();  // slot j & 1 is free again; slot (j + 1) & 1 is complete
    }
    const float2* el[NT];
    const float2* em[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int pix = min(16 * (blk * NT + t) + c16, Q - 1);
      const int im = pix / nl, il = pix - im * nl;
      el[t] = tab.El + (size_t)q * nl + il;
      em[t] = tab.Em + (size_t)q * nm + im;
    }
    // column dot over this wave's row tiles: accumulator element r of row tile m
    // pairs with chunk 4m + r, i.e. antenna 8m + 4(r >> 1) + q, component r & 1
    float gp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      gp[t] = 0.f;
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        const int m = mrow[i];
        if (m < MT) {
          const float2 a0 = cmul(el[t][(size_t)(8 * m) * nl], em[t][(size_t)(8 * m) * nm]);
          const float2 a1 = cmul(el[t][(size_t)(8 * m + 4) * nl], em[t][(size_t)(8 * m + 4) * nm]);
          gp[t] += acc[i][t][0] * a0.x + acc[i][t][1] * a0.y + acc[i][t][2] * a1.x + acc[i][t][3] * a1.y;
        }
      }
      gp[t] += __shfl_xor(gp[t], 16, 64);
      gp[t] += __shfl_xor(gp[t], 32, 64);
    }
    if (q == 0) {
#pragma unroll
      for (int t = 0; t < NT; ++t) gsum[w][16 * t + c16] = gp[t];
    }
    __syncthreads();
    if (threadIdx.x < NT * 16) {
      const int t = threadIdx.x >> 4;
      const int pix = 16 * (blk * NT + t) + (threadIdx.x & 15);
      const float g = (gsum[0][threadIdx.x] + gsum[1][threadIdx.x]) + (gsum[2][threadIdx.x] + gsum[3][threadIdx.x]);
      epi(pix, g, pix < Q);
    }
    __syncthreads();
  }
  epi.finish(blockIdx.x);
}

// ---------------------------------------------------------------------------
// Split half precision (CLSIMG_FP16, CLSIMG_BF16): the same product Y = Ut X
// on the 16 x 16 x 32 half-precision MFMA with FP32 accumulation.  Each
// operand is split into a high and a low half (v = hi + lo, lo = v - hi
// rounded again), and three products are accumulated: hi.hi + hi.lo + lo.hi.
// With FP16 (11-bit significands) the dropped lo.lo term is 2^-22 of the
// product, so the result is close to the FP32 one; with BF16 (8 bits) it is
// 2^-16.  FP16 needs the operands inside its range: Ut is scaled by a power of
// two sU (largest entry below 2^14, computed on the device) and the steering
// entries by a power of two sB (|a_p| = P^-1/2); the column dot in FP32 with
// the scaled steering entries xh + xl is multiplied by 1 / (sU sB^2) (exact).
// As in the FP32 kernel the product runs on the block triangle of Ut (blocks
// below the diagonal doubled by the preparation, zero above it; row tile m
// takes chunks 0 .. m / 2), and the B operands of a block are generated once
// per workgroup into LDS.
//
// Embedding: real position 2p + s = component s of antenna p (Ut[2p+s][2q+t]
// = Re H_pq if s == t, -Im H_pq if (s, t) = (0, 1), Im H_pq if (1, 0), with H
// the Hermitian part of U).  In K chunk c a lane of group g = lane >> 4
// supplies positions 32c + 8g + i, i.e. antennas 16c + 4g + (i >> 1) with
// both components; accumulator element r of row tile m is position
// 16m + 4g + r, i.e. antenna 8m + 2g + (r >> 1), component r & 1.
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8b __attribute__((ext_vector_type(8)));

template <bool BF>
struct Half;
template <>
struct Half<false> {
  typedef _Float16 T;
  typedef v8h V;
  __device__ static v4f mfma(V a, V b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};
template <>
struct Half<true> {
  typedef __bf16 T;
  typedef v8b V;
  __device__ static v4f mfma(V a, V b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

// power-of-two scale putting the largest |U| component just below 2^14, in
// two launches: partial maxima over kHalfScaleParts workgroups (into
// scale[1 ..]), then their maximum and the scale (scale[0])
__global__ __launch_bounds__(256) void beam_h16_scale_part_kernel(const float2* __restrict__ U, int n,
                                                                  float* __restrict__ part) {
  __shared__ float sm[4];
  float m = 0.f;
  const int stride = gridDim.x * blockDim.x;
#pragma unroll 4
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const float2 v = U[e];
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmaxf(fmaxf(sm[0], sm[1]), fmaxf(sm[2], sm[3]));
}

__global__ __launch_bounds__(64) void beam_h16_scale_kernel(float* __restrict__ scale) {
  float t = scale[1 + threadIdx.x];  // kHalfScaleParts == 64 partials
  for (int o = 32; o > 0; o >>= 1) t = fmaxf(t, __shfl_xor(t, o, 64));
  if (threadIdx.x == 0) {
    int ex = 0;
    (void)frexpf(t, &ex);  // t < 2^ex
    scale[0] = (t > 0.f && isfinite(t)) ? ldexpf(1.f, 14 - ex) : 1.f;
  }
}

static void launch_half_scale(const float2* U, int n, float* scale, hipStream_t st, hipEvent_t start = nullptr) {
  static_assert(kHalfScaleParts == 64, "one partial per lane of the final wave");
  hipExtLaunchKernelGGL(beam_h16_scale_part_kernel, dim3(kHalfScaleParts), dim3(256), 0, st, start,
                        (hipEvent_t) nullptr, 0, U, n, scale + 1);
  hipLaunchKernelGGL(beam_h16_scale_kernel, dim3(1), dim3(64), 0, st, scale);
}

// Calls f(integral_constant<int, P>) for P = 0 .. N - 1 in order.
template <class F, int... Ps>
__device__ __forceinline__ void for_each_index(F&& f, std::integer_sequence<int, Ps...>) {
  (f(std::integral_constant<int, Ps>{}), ...);
}

template <bool BF>
__device__ __forceinline__ void split_half(float v, typename Half<BF>::T& hi, typename Half<BF>::T& lo) {
  hi = (typename Half<BF>::T)v;
  lo = (typename Half<BF>::T)(v - (float)hi);
}

// fragments: [row tile m][chunk c][hi, lo][lane][8]
template <bool BF>
__global__ void beam_prep_h16_kernel(const float2* __restrict__ U, int P, int MT, int KC, const float* __restrict__ scale,
                                     typename Half<BF>::V* __restrict__ frag) {
  typedef typename Half<BF>::V V;
  const float sU = scale ? *scale : 1.f;
  const int total = 4 * big_rpw(MT) * KC * 64;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int lane = e & 63, f = e >> 6;
    const int m = f / KC, c = f - m * KC;
    const int row = 16 * m + (lane & 15), col0 = 32 * c + 8 * (lane >> 4);
    const int p = row >> 1, s = row & 1;
    V hi, lo;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int p2 = (col0 + i) >> 1, t = i & 1;
      const int ct = (col0 + i) >> 4;  // 16-column tile: below the diagonal doubled, above it zero
      float v = 0.f;
      if (m < MT && p < P && p2 < P && ct <= m) {
        const float2 x = U[p * P + p2], y = U[p2 * P + p];
        const float hr = 0.5f * (x.x + y.x), hm = 0.5f * (x.y - y.y);
        v = (s == t) ? hr : (s == 0 ? -hm : hm);
        if (ct < m) v *= 2.f;
      }
      typename Half<BF>::T h, l;
      split_half<BF>(v * sU, h, l);
      hi[i] = h;
      lo[i] = l;
    }
    frag[(size_t)(2 * f) * 64 + lane] = hi;
    frag[(size_t)(2 * f + 1) * 64 + lane] = lo;
  }
}

// Split half precision: W x = Wh xh + Wh xl + Wl xh (the lo * lo product
// dropped) on the 16 x 16 x 32 MFMA, FP32 accumulation.  Organised as the
// single-product multiplier kernel: the hi / lo B operands of every chunk of
// an NT-tile block are formed once into LDS (wave w forms tiles w, w + 4,
// ... of each chunk from the tables), the rows of a wave run in triangle
// phases with their hi / lo A fragments requested one chunk ahead (chunk 0
// of the next block behind the last one), and the column dot takes
// x = xh + xl back from LDS.
template <int RPW, int NT, bool BF, class Epi>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4 * RPW * NT + 8 * RPW + 8 * NT > 224 ? 1 : 2))) void beam_h16_kernel(
    const typename Half<BF>::V* __restrict__ frag, int MT, int KC, const float* __restrict__ scale, float sB,
    Tables tab, const int* skip, Epi epi) {
  typedef typename Half<BF>::V V;
  typedef typename Half<BF>::T T;
  typedef T V4 __attribute__((ext_vector_type(4)));
  constexpr int CMAX = 2 * RPW;
  if (skip && *skip) return;
  __shared__ float gsum[4][NT * 16];
  __shared__ V bsh[CMAX][NT][2][64];  // hi / lo B operands of every chunk, per tile and lane
  __shared__ float2 emsh[16 * CMAX];
  const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform row-tile tests
  const int Q = tab.Q, nl = tab.nl, nm = tab.nm, Pp = tab.Pp;
  const int ntiles = (Q + 15) >> 4;
  const bool row_blocks = (nl & (16 * NT - 1)) == 0;  // every block inside one image row
  const float inv = 1.f / ((scale ? *scale : 1.f) * sB * sB);
  int mrow[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) mrow[i] = 4 * i + ((i & 1) ? 3 - w : w);
  const int cend = min(KC, (MT - 1) / 2 + 1);
  int last[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) last[i] = min(mrow[i] >> 1, cend - 1);
  // hi at fragment 2 f, lo at 2 f + 1 (f = m KC + c)
  V ah[RPW], al[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const V* fr = frag + (size_t)(2 * (size_t)mrow[i] * KC) * 64 + lane;
    ah[i] = fr[0];
    al[i] = fr[64];
  }
  constexpr int GT = (NT + 3) / 4;  // tiles whose operands this wave forms
  epi.init();
  for (int blk = blockIdx.x; blk * NT < ntiles; blk += gridDim.x) {
    if (row_blocks) {
      const int im = (16 * blk * NT) / nl;
      for (int k = threadIdx.x; k < 16 * cend; k += blockDim.x) emsh[k] = tab.Em[(size_t)min(k, Pp - 1) * nm + im];
      __syncthreads();
    }
#pragma unroll
    for (int tt = 0; tt < GT; ++tt) {
      const int t = w + 4 * tt;
      if (t >= NT) continue;  // wave-uniform
      const int pw = min(16 * (blk * NT + t) + c16, Q - 1);
      const int imw = pw / nl;
      const float2* elw = tab.El + (pw - imw * nl);
      const float2* emw = tab.Em + imw;
      for (int c0 = 0; c0 < cend; c0 += 2) {
        float2 el[8], em[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int ant = min(16 * c0 + 16 * (k >> 2) + 4 * g + (k & 3), Pp - 1);  // beyond P: zero columns of Ut
          el[k] = elw[(size_t)ant * nl];
          em[k] = row_blocks ? emsh[ant] : emw[(size_t)ant * nm];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          V bh, bl;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float2 x = cmul(el[4 * h + u], em[4 * h + u]);
            T hh, ll;
            split_half<BF>(x.x * sB, hh, ll);
            bh[2 * u] = hh;
            bl[2 * u] = ll;
            split_half<BF>(x.y * sB, hh, ll);
            bh[2 * u + 1] = hh;
            bl[2 * u + 1] = ll;
          }
          bsh[c0 + h][t][0][lane] = bh;  // c0 + 1 < CMAX also when cend is odd (CMAX is even)
          bsh[c0 + h][t][1][lane] = bl;
        }
      }
    }
    __syncthreads();
    v4f acc[RPW][NT];
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[i][t] = v4f{0.f, 0.f, 0.f, 0.f};
    auto phase = [&](auto pc) {
      constexpr int P0 = decltype(pc)::value;
      const int lo = P0 == 0 ? 0 : (mrow[P0 > 0 ? P0 - 1 : 0] >> 1) + 1;
      const int hi = min(mrow[P0] >> 1, cend - 1);
      for (int c = lo; c <= hi; ++c) {
        V bh[NT], bl[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          bh[t] = bsh[c][t][0][lane];
          bl[t] = bsh[c][t][1][lane];
        }
#pragma unroll
        for (int i = P0; i < RPW; ++i) {
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            acc[i][t] = Half<BF>::mfma(ah[i], bh[t], acc[i][t]);
            acc[i][t] = Half<BF>::mfma(ah[i], bl[t], acc[i][t]);
            acc[i][t] = Half<BF>::mfma(al[i], bh[t], acc[i][t]);
          }
          const V* fr = frag + (size_t)(2 * ((size_t)mrow[i] * KC + (c < last[i] ? c + 1 : 0))) * 64 + lane;
          ah[i] = fr[0];
          al[i] = fr[64];
        }
      }
    };
    for_each_index(phase, std::make_integer_sequence<int, RPW>{});
    // the column dot with x = xh + xl, from the chunk and lane positions of
    // the single-product kernel
    float gp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      gp[t] = 0.f;
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        const int m = mrow[i];
        if (m < MT) {
          const int ln = c16 + 16 * (2 * (m & 1) + (g >> 1));
          const V4 xh = *reinterpret_cast<const V4*>(reinterpret_cast<const T*>(&bsh[m >> 1][t][0][ln]) + 4 * (g & 1));
          const V4 xl = *reinterpret_cast<const V4*>(reinterpret_cast<const T*>(&bsh[m >> 1][t][1][ln]) + 4 * (g & 1));
#pragma unroll
          for (int r = 0; r < 4; ++r) gp[t] += acc[i][t][r] * ((float)xh[r] + (float)xl[r]);
        }
      }
      gp[t] += __shfl_xor(gp[t], 16, 64);
      gp[t] += __shfl_xor(gp[t], 32, 64);
    }
    if (g == 0) {
#pragma unroll
      for (int t = 0; t < NT; ++t) gsum[w][16 * t + c16] = gp[t];
    }
    __syncthreads();  // every wave is done with bsh and emsh, and gsum is complete
    if (threadIdx.x < NT * 16) {
      const int t = threadIdx.x >> 4;
      const int pix = 16 * (blk * NT + t) + (threadIdx.x & 15);
      const float s4 = (gsum[0][threadIdx.x] + gsum[1][threadIdx.x]) + (gsum[2][threadIdx.x] + gsum[3][threadIdx.x]);
      epi(pix, s4 * inv, pix < Q);
    }
    __syncthreads();
  }
  epi.finish(blockIdx.x);
}

// ---------------------------------------------------------------------------
// Reduced precision with FP32 refinement of the decision (the multipliers of
// the host-driven loop with CLSIMG_FP16 / CLSIMG_BF16): one half-precision
// product Y = W X on the 16 x 16 x 32 MFMA with FP32 accumulation, W the
// block triangle of Ut (blocks below the diagonal doubled, as in the FP32
// kernel), gives approximate multipliers lam~_i = x~^T W~ x~, with a bound
// delta on |lam~_i - lam_i| from the rounding of the operands:
//   |x^T W x - x~^T W~ x~| <= (3u + accumulation terms) sum_jk |x_j| |W_jk| |x_k|
//                          <= (3u + ...) S / P,   S = sum |W| = sum |Ut|,
// since every real steering component is at most P^-1/2 (u = 2^-11 for FP16,
// 2^-8 for BF16).  The true minimum lies among the pixels with
// lam~_i <= min lam~ + 2 delta; those candidates are beamformed again in FP32
// and the argmin is taken over them, so the decision is the FP32 one.
//
// Fragments: [row tile m][chunk c][lane] (one 8-vector per lane), positions as
// in the split kernel; chunk c of row tile m holds the 32 columns 32c ..
// 32c + 31, zero above the diagonal block, doubled below it.  absum[b]:
// workgroup b's sum of |W| (FP32 values, summed in double, fixed order).
template <bool BF>
__global__ __launch_bounds__(256) void beam_prep_h1_kernel(const float2* __restrict__ U, int P, int MT, int KC,
                                                           const float* __restrict__ scale,
                                                           typename Half<BF>::V* __restrict__ frag,
                                                           double* __restrict__ absum, int* __restrict__ count) {
  typedef typename Half<BF>::V V;
  __shared__ double sh[4];
  const float sU = scale ? *scale : 1.f;
  const int total = 4 * big_rpw(MT) * KC * 64;
  if (blockIdx.x == 0 && threadIdx.x == 0 && count) *count = 0;  // candidates of the coming selection
  double acc = 0.0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    const int lane = e & 63, f = e >> 6;
    const int m = f / KC, c = f - m * KC;
    const int row = 16 * m + (lane & 15), col0 = 32 * c + 8 * (lane >> 4);
    const int p = row >> 1, s = row & 1;
    V hv;
    float a = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int col = col0 + i, p2 = col >> 1, t = i & 1;
      const int ct = col >> 4;  // 16-column tile
      float v = 0.f;
      if (m < MT && p < P && p2 < P && ct <= m) {
        const float2 x = U[p * P + p2], y = U[p2 * P + p];
        const float hr = 0.5f * (x.x + y.x), hm = 0.5f * (x.y - y.y);
        v = (s == t) ? hr : (s == 0 ? -hm : hm);
        if (ct < m) v *= 2.f;
      }
      a += fabsf(v);
      hv[i] = (typename Half<BF>::T)(v * sU);
    }
    acc += (double)a;
    frag[(size_t)f * 64 + lane] = hv;
  }
  const double tot = block_sum_d(acc, sh);
  if (threadIdx.x == 0) absum[blockIdx.x] = tot;
}

// The approximate multipliers: lam~ in lam[] (+inf for free pixels) and one
// argmin key per workgroup in part[].
struct BeamLambdaApprox {
  const uint8_t* state;
  uint64_t* part;
  float* lam;
  uint64_t best;
  __device__ void init() { best = ~0ull; }
  __device__ void operator()(int pix, float g, bool ok) {
    if (ok) {
      const uint8_t s = state[pix];
      float l = __builtin_inff();
      if (s != 1) {
        l = (s == 0) ? g : -g;
        const uint64_t key = ((uint64_t)ordered_bits(l) << 32) | (uint32_t)pix;
        best = key < best ? key : best;
      }
      lam[pix] = l;
    }
  }
  __device__ void finish(int blk) {
    __shared__ uint64_t sh[4];
    const uint64_t m = block_min_u64(best, sh);
    if (threadIdx.x == 0) part[blk] = m;
  }
};

// Single product on the half MFMA, block-triangular; waves own row tiles
// m = 4i + w (even i) or 4i + 3 - w (odd i) as in the FP32 kernel, and row
// tile m runs chunks 0 .. m / 2.  Per block of NT = 4 pixel tiles the B
// operands of every chunk the triangle touches (at most 2 RPW chunks of 16
// antennas) are formed once, wave w forming tile w's from the tables (the
// block's column of the m table staged in LDS first when the block lies in
// one image row), and stay in LDS for the whole block: the chunk loop has
// no barrier.  The rows of a wave are sorted by m, so the chunks fall into
// phases p = 0 .. RPW - 1 in which exactly rows p .. RPW - 1 are active;
// each phase is its own loop with a fixed set of rows.  A fragments stream
// from global memory one chunk ahead (row i's fragment of chunk c + 1, or of
// chunk 0 of the next block behind its last chunk, is requested right behind
// its MFMAs of chunk c, in a fixed order, so the waits count exactly), and
// the column dot takes the same rounded steering components back from LDS:
// lam~ = x~^T W~ x~, every operand rounded once.
template <int RPW, bool BF, class Epi>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void beam_h1_kernel(
    const typename Half<BF>::V* __restrict__ frag, int MT, int KC, const float* __restrict__ scale, float sB,
    Tables tab, const int* skip, Epi epi) {
  typedef typename Half<BF>::V V;
  typedef typename Half<BF>::T T;
  typedef T V4 __attribute__((ext_vector_type(4)));
  constexpr int NT = 4, CMAX = 2 * RPW;
  if (skip && *skip) return;
  __shared__ float gsum[4][NT * 16];
  __shared__ V bsh[CMAX][NT][64];
  __shared__ float2 emsh[16 * CMAX];
  const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform row-tile tests
  const int Q = tab.Q, nl = tab.nl, nm = tab.nm, Pp = tab.Pp;
  const int ntiles = (Q + 15) >> 4;
  const bool row_blocks = (nl & (16 * NT - 1)) == 0;  // every block inside one image row
  const float inv = 1.f / ((scale ? *scale : 1.f) * sB * sB);
  int mrow[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) mrow[i] = 4 * i + ((i & 1) ? 3 - w : w);
  // chunks the triangle touches: 0 .. (MT - 1) / 2 (at most CMAX)
  const int cend = min(KC, (MT - 1) / 2 + 1);
  // each row's last chunk: its diagonal chunk (rows from MT on are zero
  // fragments, row tiles up to 4 RPW being allocated); behind it the row
  // requests chunk 0 again, the first one of the next block
  int last[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) last[i] = min(mrow[i] >> 1, cend - 1);
  V a[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) a[i] = frag[(size_t)mrow[i] * KC * 64 + lane];
  epi.init();
  for (int blk = blockIdx.x; blk * NT < ntiles; blk += gridDim.x) {
    if (row_blocks) {
      const int im = (16 * blk * NT) / nl;
      for (int k = threadIdx.x; k < 16 * cend; k += blockDim.x) emsh[k] = tab.Em[(size_t)min(k, Pp - 1) * nm + im];
      __syncthreads();
    }
    {
      const int pw = min(16 * (blk * NT + w) + c16, Q - 1);
      const int imw = pw / nl;
      const float2* elw = tab.El + (pw - imw * nl);
      const float2* emw = tab.Em + imw;
      // two chunks per round, all table reads issued before use
      for (int c0 = 0; c0 < cend; c0 += 2) {
        float2 el[8], em[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int ant = min(16 * c0 + 16 * (k >> 2) + 4 * g + (k & 3), Pp - 1);  // beyond P: zero columns of W
          el[k] = elw[(size_t)ant * nl];
          em[k] = row_blocks ? emsh[ant] : emw[(size_t)ant * nm];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          V bh;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float2 x = cmul(el[4 * h + u], em[4 * h + u]);
            bh[2 * u] = (T)(x.x * sB);
            bh[2 * u + 1] = (T)(x.y * sB);
          }
          bsh[c0 + h][w][lane] = bh;  // c0 + 1 < CMAX also when cend is odd (CMAX is even)
        }
      }
    }
    __syncthreads();
    v4f acc[RPW][NT];
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[i][t] = v4f{0.f, 0.f, 0.f, 0.f};
    auto phase = [&](auto pc) {
      constexpr int P0 = decltype(pc)::value;
      const int lo = P0 == 0 ? 0 : (mrow[P0 > 0 ? P0 - 1 : 0] >> 1) + 1;
      const int hi = min(mrow[P0] >> 1, cend - 1);
      for (int c = lo; c <= hi; ++c) {
        V bh[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) bh[t] = bsh[c][t][lane];
#pragma unroll
        for (int i = P0; i < RPW; ++i) {
#pragma unroll
          for (int t = 0; t < NT; ++t) acc[i][t] = Half<BF>::mfma(a[i], bh[t], acc[i][t]);
          a[i] = frag[((size_t)mrow[i] * KC + (c < last[i] ? c + 1 : 0)) * 64 + lane];
        }
      }
    };
    for_each_index(phase, std::make_integer_sequence<int, RPW>{});
    // lane (c16, g) holds rows 4g .. 4g + 3 of row tile m: antennas 8m + 2g
    // and 8m + 2g + 1 (real, imaginary), which sit in chunk m / 2 at lane
    // c16 + 16 (2 (m & 1) + g / 2), halves 4 (g & 1) .. 4 (g & 1) + 3
    float gp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      gp[t] = 0.f;
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        const int m = mrow[i];
        if (m < MT) {
          const T* xs = reinterpret_cast<const T*>(&bsh[m >> 1][t][c16 + 16 * (2 * (m & 1) + (g >> 1))]);
          const V4 x = *reinterpret_cast<const V4*>(xs + 4 * (g & 1));
          gp[t] += acc[i][t][0] * (float)x[0] + acc[i][t][1] * (float)x[1] + acc[i][t][2] * (float)x[2] +
                   acc[i][t][3] * (float)x[3];
        }
      }
      gp[t] += __shfl_xor(gp[t], 16, 64);
      gp[t] += __shfl_xor(gp[t], 32, 64);
    }
    if (g == 0) {
#pragma unroll
      for (int t = 0; t < NT; ++t) gsum[w][16 * t + c16] = gp[t];
    }
    __syncthreads();  // every wave is done with bsh and emsh, and gsum is complete
    if (threadIdx.x < NT * 16) {
      const int t = threadIdx.x >> 4;
      const int pix = 16 * (blk * NT + t) + (threadIdx.x & 15);
      const float s4 = (gsum[0][threadIdx.x] + gsum[1][threadIdx.x]) + (gsum[2][threadIdx.x] + gsum[3][threadIdx.x]);
      epi(pix, s4 * inv, pix < Q);
    }
    __syncthreads();
  }
  epi.finish(blockIdx.x);
}

// Candidates of the FP32 refinement: every workgroup reduces the argmin keys
// (min lam~) and the |W| partials (S) in a fixed order, forms
//   delta = coef S + coef_abs S_abs,   threshold = min lam~ + 2 delta
// (in double), and appends the pixels of its slice with lam~ <= threshold to
// cand[] (order immaterial: the FP32 argmin key carries the pixel index).
// *count ends as the number of candidates, possibly beyond cap.
__global__ __launch_bounds__(256) void beam_cand_kernel(const uint64_t* __restrict__ keys, int nkeys,
                                                        const double* __restrict__ absum, int nabs, double coef,
                                                        const float* __restrict__ lam, int Q, const int* skip,
                                                        int* __restrict__ cand, int cap, int* __restrict__ count) {
  __shared__ uint64_t shk[4];
  __shared__ double shs[4];
  if (skip && *skip) return;
  // this thread's first four multipliers, the keys and the partials, all
  // requested before the reductions
  constexpr int L4 = 4;
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
  float l4[L4];
#pragma unroll
  for (int u = 0; u < L4; ++u) l4[u] = i0 + u * stride < Q ? lam[i0 + u * stride] : 0.f;
  uint64_t m = ~0ull;
  int i = threadIdx.x;
  for (; i + 3 * (int)blockDim.x < nkeys; i += 4 * blockDim.x) {
    uint64_t k4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) k4[u] = keys[i + u * blockDim.x];
#pragma unroll
    for (int u = 0; u < 4; ++u) m = k4[u] < m ? k4[u] : m;
  }
  for (; i < nkeys; i += blockDim.x) m = keys[i] < m ? keys[i] : m;
  double sa = 0.0;
  for (int j = threadIdx.x; j < nabs; j += blockDim.x) sa += absum[j];
  m = block_min_u64(m, shk);
  const double S = block_sum_d(sa, shs);
  if (m == ~0ull) return;  // no active pixel
  const double lmin = (double)from_ordered_bits((uint32_t)(m >> 32));
  const double thr = lmin + 2.0 * coef * S;
#pragma unroll
  for (int u = 0; u < L4; ++u) {
    const int ii = i0 + u * stride;
    if (ii < Q && (double)l4[u] <= thr) {
      const int k = atomicAdd(count, 1);
      if (k < cap) cand[k] = ii;
    }
  }
  for (int ii = i0 + L4 * stride; ii < Q; ii += stride) {
    const float l = lam[ii];
    if ((double)l <= thr) {
      const int k = atomicAdd(count, 1);
      if (k < cap) cand[k] = ii;
    }
  }
}

bool beam_fits(int P) { return pad_p(P) / 8 <= kBeamMaxMT; }

constexpr int kBigMaxRPW = 9;  // up to 36 row tiles: P <= 288
// Grid cap of the block-triangular beamformers (FP32, split half, one
// product): four workgroups per CU, each looping over pixel blocks.  At 288
// antennas and 512^2 against one workgroup per block: FP32 1059 -> 1042 us,
// split FP16 376 -> 360 us, one product 162 -> 151 us per launch; caps of 512
// and 2048 measured within 2 % of this one, 256 took the one-product kernel
// to 234 us.  Kernels that leave one key per workgroup are reduced over this
// many keys.
constexpr int kBigMaxWorkgroups = 1024;
bool beam_big_fits(int P) { return big_rpw(pad_p(P) / 8) <= kBigMaxRPW; }

size_t beam_big_frag_floats(int P) {
  const int MT = pad_p(P) / 8;
  return (size_t)4 * big_rpw(MT) * 4 * MT * 64;
}

int beam_big_grid(int P, int Q, int nt) {
  nt = big_nt_or(nt, big_rpw(pad_p(P) / 8));
  const int nblk = ((Q + 15) / 16 + nt - 1) / nt;
  return nblk < 1 ? 1 : (nblk > kBigMaxWorkgroups ? kBigMaxWorkgroups : nblk);
}

int beam_grid(int Q) {
  const int ntiles = (Q + 15) / 16;
  int g = (ntiles + kBeamWaves - 1) / kBeamWaves;
  return g < 1 ? 1 : (g > 2048 ? 2048 : g);
}

int beam_grid_batched(int Q, int tiles) {
  const int ntiles = (Q + 15) / 16;
  const int per = kBeamWaves * (tiles < 1 ? 1 : tiles);
  int g = (ntiles + per - 1) / per;
  return g < 1 ? 1 : (g > 2048 ? 2048 : g);
}

int beam_batch_tiles(int n, int Q) {
  int t = 16;
  while (t > 1 && (long long)n * beam_grid_batched(Q, t) < 1024) t >>= 1;
  return t;
}

hipError_t launch_beam_prep(const float2* U, int P, float* frag, hipStream_t st, Stamps ts) {
  const int MT = pad_p(P) / 8;
  const int n = 2 * MT * (MT + 1) * 64;
  hipExtLaunchKernelGGL(beam_prep_kernel, dim3((n + 255) / 256), dim3(256), 0, st, ts.start, ts.stop, 0, U, P, MT,
                        frag);
  return hipGetLastError();
}

template <class Epi>
static hipError_t launch_beam(const float* frag, const float2* U, int P, const Tables& tab, const int* skip,
                              Epi epi, hipStream_t st, Stamps ts = {}) {
  const dim3 g(beam_grid(tab.Q)), b(64 * kBeamWaves);
  switch (tab.Pp / 8) {
    case 1: hipExtLaunchKernelGGL((beam_kernel<1, Epi>), g, b, 0, st, ts.start, ts.stop, 0, frag, U, P, tab, skip, epi); break;
    case 2: hipExtLaunchKernelGGL((beam_kernel<2, Epi>), g, b, 0, st, ts.start, ts.stop, 0, frag, U, P, tab, skip, epi); break;
    case 3: hipExtLaunchKernelGGL((beam_kernel<3, Epi>), g, b, 0, st, ts.start, ts.stop, 0, frag, U, P, tab, skip, epi); break;
    case 4: hipExtLaunchKernelGGL((beam_kernel<4, Epi>), g, b, 0, st, ts.start, ts.stop, 0, frag, U, P, tab, skip, epi); break;
    case 5: hipExtLaunchKernelGGL((beam_kernel<5, Epi>), g, b, 0, st, ts.start, ts.stop, 0, frag, U, P, tab, skip, epi); break;
    case 6: hipExtLaunchKernelGGL((beam_kernel<6, Epi>), g, b, 0, st, ts.start, ts.stop, 0, frag, U, P, tab, skip, epi); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_beam_prep_full(const float2* U, int P, float* frag, hipStream_t st, Stamps ts) {
  const int MT = pad_p(P) / 8;
  const size_t n = beam_big_frag_floats(P);
  int g = (int)((n + 255) / 256);
  if (g > 4096) g = 4096;
  hipExtLaunchKernelGGL(beam_prep_full_kernel, dim3(g), dim3(256), 0, st, ts.start, ts.stop, 0, U, P, MT, frag);
  return hipGetLastError();
}

template <class Epi>
static hipError_t launch_big(const float* frag, const Tables& tab, const int* skip, Epi epi, hipStream_t st,
                             Stamps ts = {}, int nt = 0) {
  const int MT = tab.Pp / 8, rpw = big_rpw(MT);
  nt = big_nt_or(nt, rpw);
  const dim3 g(beam_big_grid(tab.Pp, tab.Q, nt)), b(256);
  switch (10 * rpw + nt / 4) {  // nt 2, 4, 8 -> 0, 1, 2
#define BIG_CASE(R, N)                                                                                         \
  case 10 * R + N / 4:                                                                                         \
    hipExtLaunchKernelGGL((beam_big_kernel<R, N, Epi>), g, b, 0, st, ts.start, ts.stop, 0, frag, MT, tab, skip, \
                          epi);                                                                                \
    break;
#define BIG_RPW(R) BIG_CASE(R, 2) BIG_CASE(R, 4) BIG_CASE(R, 8)
#define BIG_RPW_LARGE(R) BIG_CASE(R, 2) BIG_CASE(R, 4)
    BIG_RPW(1)
    BIG_RPW(2)
    BIG_RPW(3)
    BIG_RPW(4)
    BIG_RPW(5)
    BIG_RPW(6)
    BIG_RPW_LARGE(7)
    BIG_RPW_LARGE(8)
    BIG_RPW_LARGE(9)
#undef BIG_RPW_LARGE
#undef BIG_RPW
#undef BIG_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_beam_big(int kind, const float* frag, const Tables& tab, const int* skip, float* out, float* eps,
                           float eps_scale, double C, double kb, float scale, const uint8_t* state, uint64_t* part,
                           hipStream_t st, Stamps ts, int nt, const float* lam_scale) {
  switch (kind) {
    case 0: return launch_big(frag, tab, skip, BeamMF{out, eps, eps_scale}, st, ts, nt);
    case 1: return launch_big(frag, tab, skip, BeamMVDR{out, C, kb}, st, ts, nt);
    case 2: return launch_big(frag, tab, skip, BeamStore{out, scale}, st, ts, nt);
    default: return launch_big(frag, tab, skip, BeamLambda{state, part, lam_scale, 0}, st, ts, nt);
  }
}

// ---- split half precision ----
int beam_h16_chunks(int P) { return (2 * pad_p(P) + 31) / 32; }

// 16-pixel tiles per workgroup of the split kernel: the hi / lo operands of a
// block (2 RPW chunks x NT tiles x 2 KiB) stay in LDS, so eight tiles only up
// to 4 row tiles per wave; two tiles by default (two workgroups per CU up to
// 9 row tiles per wave)
__host__ __device__ constexpr bool h16_nt_ok(int nt, int rpw) { return nt == 2 || nt == 4 || (nt == 8 && rpw <= 4); }
__host__ __device__ inline int h16_nt_or(int nt, int rpw) { return h16_nt_ok(nt, rpw) ? nt : 2; }

bool beam_tiles_offered(bool half, int nt, int rpw) { return half ? h16_nt_ok(nt, rpw) : big_nt_ok(nt, rpw); }

size_t beam_h16_frag_bytes(int P) {
  const int MT = pad_p(P) / 8;
  return (size_t)4 * big_rpw(MT) * beam_h16_chunks(P) * 2 * 64 * 16;
}

template <bool BF, class Epi>
static hipError_t launch_h16(const void* frag, const float* scale, const Tables& tab, const int* skip, Epi epi,
                             hipStream_t st, Stamps ts = {}, int nt = 0) {
  typedef typename Half<BF>::V V;
  const int MT = tab.Pp / 8, KC = beam_h16_chunks(tab.Pp), rpw = big_rpw(MT);
  nt = h16_nt_or(nt, rpw);
  // steering entries scaled towards unit magnitude (|a_p| = P^-1/2): a power of two
  int ex = 0;
  (void)frexpf(sqrtf((float)tab.Pp), &ex);
  const float sB = BF ? 1.f : ldexpf(1.f, ex - 1);
  const V* f = static_cast<const V*>(frag);
  const dim3 g(beam_big_grid(tab.Pp, tab.Q, nt)), b(256);
  switch (10 * rpw + nt / 4) {
#define H16_CASE(R, N)                                                                                             \
  case 10 * R + N / 4:                                                                                             \
    hipExtLaunchKernelGGL((beam_h16_kernel<R, N, BF, Epi>), g, b, 0, st, ts.start, ts.stop, 0, f, MT, KC, scale, sB, \
                          tab, skip, epi);                                                                         \
    break;
#define H16_RPW(R) H16_CASE(R, 2) H16_CASE(R, 4) H16_CASE(R, 8)
#define H16_RPW_LARGE(R) H16_CASE(R, 2) H16_CASE(R, 4)
    H16_RPW(1)
    H16_RPW(2)
    H16_RPW(3)
    H16_RPW(4)
    H16_RPW_LARGE(5)
    H16_RPW_LARGE(6)
    H16_RPW_LARGE(7)
    H16_RPW_LARGE(8)
    H16_RPW_LARGE(9)
#undef H16_RPW_LARGE
#undef H16_RPW
#undef H16_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_beam_prep_h16(const float2* U, int P, bool bf16, void* frag, float* scale, hipStream_t st,
                                Stamps ts) {
  const int MT = pad_p(P) / 8, KC = beam_h16_chunks(P);
  if (!bf16) {  // the scale pass comes first: it takes the start stamp
    launch_half_scale(U, P * P, scale, st, ts.start);
    ts.start = nullptr;
  }
  const int total = 4 * big_rpw(MT) * KC * 64;
  const int g = std::min((total + 255) / 256, 4096);
  if (bf16)
    hipExtLaunchKernelGGL(beam_prep_h16_kernel<true>, dim3(g), dim3(256), 0, st, ts.start, ts.stop, 0, U, P, MT, KC,
                          (const float*)nullptr, static_cast<v8b*>(frag));
  else
    hipExtLaunchKernelGGL(beam_prep_h16_kernel<false>, dim3(g), dim3(256), 0, st, ts.start, ts.stop, 0, U, P, MT, KC,
                          (const float*)scale, static_cast<v8h*>(frag));
  return hipGetLastError();
}

hipError_t launch_beam_h16(int kind, bool bf16, const void* frag, const float* scale, const Tables& tab,
                           const int* skip, float* out, float* eps, float eps_scale, double C, double kb, float sc,
                           const uint8_t* state, uint64_t* part, hipStream_t st, Stamps ts, int nt) {
  const float* s = bf16 ? nullptr : scale;
  switch (kind) {
    case 0:
      return bf16 ? launch_h16<true>(frag, s, tab, skip, BeamMF{out, eps, eps_scale}, st, ts, nt)
                  : launch_h16<false>(frag, s, tab, skip, BeamMF{out, eps, eps_scale}, st, ts, nt);
    case 1:
      return bf16 ? launch_h16<true>(frag, s, tab, skip, BeamMVDR{out, C, kb}, st, ts, nt)
                  : launch_h16<false>(frag, s, tab, skip, BeamMVDR{out, C, kb}, st, ts, nt);
    case 2:
      return bf16 ? launch_h16<true>(frag, s, tab, skip, BeamStore{out, sc}, st, ts, nt)
                  : launch_h16<false>(frag, s, tab, skip, BeamStore{out, sc}, st, ts, nt);
    default:
      return bf16 ? launch_h16<true>(frag, s, tab, skip, BeamLambda{state, part, nullptr, 0}, st, ts, nt)
                  : launch_h16<false>(frag, s, tab, skip, BeamLambda{state, part, nullptr, 0}, st, ts, nt);
  }
}

// ---- reduced precision with FP32 refinement of the decision ----
static float h1_sB(int Pp, bool bf16) {
  int ex = 0;
  (void)frexpf(sqrtf((float)Pp), &ex);
  return bf16 ? 1.f : ldexpf(1.f, ex - 1);
}

size_t beam_h1_frag_bytes(int P) {
  const int MT = pad_p(P) / 8;
  return (size_t)4 * big_rpw(MT) * beam_h16_chunks(P) * 64 * 16;
}

double beam_h1_delta_coef(int P, bool bf16) {
  // 3u for the three rounded operands (x~ on both sides, W~), accumulation
  // of up to 8 Pp + 64 FP32 terms over the half and the FP32 evaluations
  // (2^-24 each), FP16 subnormals (at most 2^-25 absolute per scaled entry,
  // far below u |v| for the entries that matter; covered by the factor 1.5 of
  // the whole bound)
  const double u = bf16 ? std::ldexp(1.0, -8) : std::ldexp(1.0, -11);
  const int Pp = pad_p(P);
  return 1.5 * (3.0 * u + (8.0 * Pp + 64.0) * std::ldexp(1.0, -24)) / (double)P;
}

hipError_t launch_beam_lambda_refined(const float2* E, int P, bool bf16, const Tables& tab, const int* skip,
                                      const uint8_t* state, void* frag, float* scale, double* absum, int nabs,
                                      uint64_t* keys, float* lam, int* cand, int cap, int* count, hipStream_t st,
                                      int nt, Stamps ts) {
  const int MT = pad_p(P) / 8, KC = beam_h16_chunks(P), rpw = big_rpw(MT);
  if (!bf16) launch_half_scale(E, P * P, scale, st);
  if (bf16)
    hipLaunchKernelGGL(beam_prep_h1_kernel<true>, dim3(nabs), dim3(256), 0, st, E, P, MT, KC, (const float*)nullptr,
                       static_cast<v8b*>(frag), absum, count);
  else
    hipLaunchKernelGGL(beam_prep_h1_kernel<false>, dim3(nabs), dim3(256), 0, st, E, P, MT, KC, (const float*)scale,
                       static_cast<v8h*>(frag), absum, count);
  // four 16-pixel tiles per workgroup (one per wave for the operand
  // generation), two waves per SIMD
  (void)nt;
  nt = 4;
  const float sB = h1_sB(tab.Pp, bf16);
  const dim3 g(beam_big_grid(tab.Pp, tab.Q, nt)), b(256);
  const BeamLambdaApprox epi{state, keys, lam, 0};
  const float* sc = bf16 ? nullptr : scale;
#define H1_RPW(R)                                                                                              \
  case R:                                                                                                      \
    if (bf16)                                                                                                  \
      hipExtLaunchKernelGGL((beam_h1_kernel<R, true, BeamLambdaApprox>), g, b, 0, st, ts.start, ts.stop, 0,     \
                            static_cast<const v8b*>(frag), MT, KC, sc, sB, tab, skip, epi);                    \
    else                                                                                                       \
      hipExtLaunchKernelGGL((beam_h1_kernel<R, false, BeamLambdaApprox>), g, b, 0, st, ts.start, ts.stop, 0,    \
                            static_cast<const v8h*>(frag), MT, KC, sc, sB, tab, skip, epi);                    \
    break;
  switch (rpw) {
    H1_RPW(1)
    H1_RPW(2)
    H1_RPW(3)
    H1_RPW(4)
    H1_RPW(5)
    H1_RPW(6)
    H1_RPW(7)
    H1_RPW(8)
    H1_RPW(9)
    default: return hipErrorInvalidValue;
  }
#undef H1_RPW
  hipLaunchKernelGGL(beam_cand_kernel, dim3(256), dim3(256), 0, st, (const uint64_t*)keys, (int)g.x,
                     (const double*)absum, nabs, beam_h1_delta_coef(P, bf16), (const float*)lam, tab.Q, skip, cand,
                     cap, count);
  return hipGetLastError();
}

hipError_t launch_beam_accumulate(const float2* U, int P, const Tables& tab, const int* skip, float* sum,
                                  float* sumsq, float scale, int first, int prec, float* frag_big, void* frag_half,
                                  float* hscale, hipStream_t st, int nt) {
  const BeamAcc epi{sum, sumsq, scale, first};
  if (prec != 0) {  // split half precision
    const bool bf = prec == 2;
    hipError_t e = launch_beam_prep_h16(U, P, bf, frag_half, hscale, st);
    if (e != hipSuccess) return e;
    return bf ? launch_h16<true>(frag_half, nullptr, tab, skip, epi, st, {}, nt)
              : launch_h16<false>(frag_half, hscale, tab, skip, epi, st, {}, nt);
  }
  if (beam_fits(P)) return launch_beam(nullptr, U, P, tab, skip, epi, st);
  hipError_t e = launch_beam_prep_full(U, P, frag_big, st);
  if (e != hipSuccess) return e;
  return launch_big(frag_big, tab, skip, epi, st, {}, nt);
}

hipError_t launch_beam_mf(const float* frag, const float2* U, int P, const Tables& tab, float* mf, float* eps,
                          float eps_scale, hipStream_t st, Stamps ts) {
  return launch_beam(frag, U, P, tab, nullptr, BeamMF{mf, eps, eps_scale}, st, ts);
}

hipError_t launch_beam_mvdr(const float* frag, const float2* U, int P, const Tables& tab, float* gamma, double C,
                            double kb_coef, hipStream_t st) {
  return launch_beam(frag, U, P, tab, nullptr, BeamMVDR{gamma, C, kb_coef}, st);
}

hipError_t launch_beam_store(const float* frag, const float2* U, int P, const Tables& tab, float* out,
                             float scale, hipStream_t st) {
  return launch_beam(frag, U, P, tab, nullptr, BeamStore{out, scale}, st);
}

hipError_t launch_beam_lambda_batch(const BeamLamItem* items, int nreq, int bpr, int P, hipStream_t st) {
  const dim3 g(nreq * bpr), b(64 * kBeamWaves);
  switch (pad_p(P) / 8) {
    case 1: hipLaunchKernelGGL(beam_lambda_batch_kernel<1>, g, b, 0, st, items, bpr); break;
    case 2: hipLaunchKernelGGL(beam_lambda_batch_kernel<2>, g, b, 0, st, items, bpr); break;
    case 3: hipLaunchKernelGGL(beam_lambda_batch_kernel<3>, g, b, 0, st, items, bpr); break;
    case 4: hipLaunchKernelGGL(beam_lambda_batch_kernel<4>, g, b, 0, st, items, bpr); break;
    case 5: hipLaunchKernelGGL(beam_lambda_batch_kernel<5>, g, b, 0, st, items, bpr); break;
    case 6: hipLaunchKernelGGL(beam_lambda_batch_kernel<6>, g, b, 0, st, items, bpr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_beam_setup_batch(const BeamSetItem* items, int nreq, int bpr, int P, hipStream_t st) {
  const dim3 g(nreq * bpr, 2), b(64 * kBeamWaves);
  switch (pad_p(P) / 8) {
    case 1: hipLaunchKernelGGL(beam_setup_batch_kernel<1>, g, b, 0, st, items, bpr); break;
    case 2: hipLaunchKernelGGL(beam_setup_batch_kernel<2>, g, b, 0, st, items, bpr); break;
    case 3: hipLaunchKernelGGL(beam_setup_batch_kernel<3>, g, b, 0, st, items, bpr); break;
    case 4: hipLaunchKernelGGL(beam_setup_batch_kernel<4>, g, b, 0, st, items, bpr); break;
    case 5: hipLaunchKernelGGL(beam_setup_batch_kernel<5>, g, b, 0, st, items, bpr); break;
    case 6: hipLaunchKernelGGL(beam_setup_batch_kernel<6>, g, b, 0, st, items, bpr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_beam_lambda(const float* frag, const float2* U, int P, const Tables& tab, const int* skip,
                              const uint8_t* state, uint64_t* part, const float* scale, hipStream_t st) {
  return launch_beam(frag, U, P, tab, skip, BeamLambda{state, part, scale, 0}, st);
}

}  // namespace clsimg
