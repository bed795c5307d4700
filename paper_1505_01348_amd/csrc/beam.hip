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
  __device__ void finish(int blk) {
    __shared__ uint64_t sh[kBeamWaves];
    const uint64_t m = block_min_u64(best, sh);
    if (threadIdx.x == 0) part[blk] = m;
  }
};

// Fragments built from U by the whole workgroup: the (m, j) pairs of chunks
// 2j, 2j + 1 of row tile m (same values as beam_prep_kernel) are dealt round
// robin to the waves, written to LDS and then read back by every wave.  For
// row tile m the lane's row is antenna 8m + 4((c16 >> 1) & 1) + (c16 >> 2),
// component c16 & 1; the pair shares column antenna 4j + q and takes the two
// components of the same Hermitian-part entry.
template <int MT>
__device__ __forceinline__ void beam_frags_from_u(const float2* __restrict__ U, int P, float* sfr, float* fa) {
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
    xv[i] = U[p * P + p2];
    yv[i] = U[p2 * P + p];
  }
#pragma unroll
  for (int i = 0; i < PPW; ++i) {
    if (w + kBeamWaves * i < NPAIR) {
      const int m = mm[i], j = jj[i];
      const bool live = 8 * m + pr0 < P && 4 * j + q < P;
      const float d = (j >> 1) < m ? 2.f : 1.f;  // chunks 2j, 2j+1 lie in column tile j >> 1
      const float hr = live ? 0.5f * d * (xv[i].x + yv[i].x) : 0.f;
      const float hi = live ? 0.5f * d * (xv[i].y - yv[i].y) : 0.f;
      const int f = 2 * m * (m + 1) + 2 * j;
      sfr[f * 64 + lane] = s1 ? hi : hr;
      sfr[(f + 1) * 64 + lane] = s1 ? hr : -hi;
    }
  }
  __syncthreads();
#pragma unroll
  for (int f = 0; f < NFR; ++f) fa[f] = sfr[f * 64 + lane];
}

template <int MT, class Epi>
__device__ __forceinline__ void beam_body(const float* __restrict__ frag, const float2* __restrict__ U, int P,
                                          const Tables& tab, const int* skip, Epi& epi, int blk, int nblk) {
  constexpr int KS = 4 * MT;             // 4-row chunks of the embedding
  constexpr int NFR = 2 * MT * (MT + 1);  // fragments of the lower block triangle
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
  const int Q = tab.Q, nl = tab.nl, nm = tab.nm;
  const int ntiles = (Q + 15) >> 4;
  const int nwav = nblk * kBeamWaves;
  // table entries of antennas 4 j + q for this lane's pixel of a tile; the
  // loads of the next tile are issued before the current one is multiplied
  float2 te[KS / 2], tm[KS / 2];
  auto load_tables = [&](int tile) {
    const int pix = min(16 * tile + c16, Q - 1);
    const int im = pix / nl, il = pix - im * nl;
    const float2* el = tab.El + (size_t)q * nl + il;
    const float2* em = tab.Em + (size_t)q * nm + im;
#pragma unroll
    for (int j = 0; j < KS / 2; ++j) {
      te[j] = el[(size_t)4 * j * nl];
      tm[j] = em[(size_t)4 * j * nm];
    }
  };
  int tile = blk * kBeamWaves + (threadIdx.x >> 6);
  if (tile < ntiles) load_tables(tile);
  float fa[NFR];
  if (U) {
    __shared__ float sfr[NFR * 64];
    beam_frags_from_u<MT>(U, P, sfr, fa);
  } else {
#pragma unroll
    for (int f = 0; f < NFR; ++f) fa[f] = frag[f * 64 + lane];
  }
  epi.init();
  for (; tile < ntiles; tile += nwav) {
    const int pix = 16 * tile + c16;
    float b[KS];
#pragma unroll
    for (int j = 0; j < KS / 2; ++j) {
      const float2 a = cmul(te[j], tm[j]);
      b[2 * j] = a.x;
      b[2 * j + 1] = a.y;
    }
    if (tile + nwav < ntiles) load_tables(tile + nwav);
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
    epi(pix, g, pix < Q && q == 0);
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

// ---------------------------------------------------------------------------
// Larger arrays (P > 48): the fragments of the whole Ut no longer fit in
// registers, so the product is organised like a GEMM.  A workgroup takes NT
// 16-pixel tiles (two or four); wave w owns the row tiles m = w, w + 4, ...
// (RPW of them, padded rows are zero) and streams their fragments from L2
// (prepared once per call by beam_prep_full_kernel, same row permutation as
// above, full matrix, no doubling) while it generates the B operands of the
// four pixel tiles from the tables, one complex product per two 4-row
// chunks.  After the K loop the column dot needs the lane's entries of its own
// row tiles again: they are recomputed from the tables (two complex products
// per row tile and pixel tile).  The four waves' partial sums meet in LDS.
__host__ __device__ inline int big_rpw(int MT) { return (MT + 3) / 4; }
// 16-pixel tiles per workgroup (measured: two for up to 16 row tiles, where
// more workgroups hide the load latency, four for longer K loops, where the
// fragment loads are shared by more MFMAs)
__host__ __device__ constexpr int big_nt(int rpw) { return rpw <= 4 ? 2 : 4; }
// loads of the next chunk pair issued before the current pair's MFMAs while
// the registers allow it (short K loops, i.e. up to 16 row tiles)
__host__ __device__ constexpr bool big_prefetch(int rpw) { return rpw <= 4; }

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
    if (m < MT && p < P && p2 < P) {
      const float2 x = U[p * P + p2], y = U[p2 * P + p];
      const float hr = 0.5f * (x.x + y.x), hi = 0.5f * (x.y - y.y);
      v = (s == t) ? hr : (s == 0 ? -hi : hi);
    }
    frag[e] = v;
  }
}

template <int RPW, class Epi>
__global__ __launch_bounds__(256) void beam_big_kernel(const float* __restrict__ frag, int MT, Tables tab,
                                                       const int* skip, Epi epi) {
  constexpr int NT = big_nt(RPW);
  constexpr bool kPrefetch = big_prefetch(RPW);
  if (skip && *skip) return;
  __shared__ float gsum[4][NT * 16];
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
  const int w = threadIdx.x >> 6;
  const int KS = 4 * MT;
  const int Q = tab.Q, nl = tab.nl, nm = tab.nm;
  const int ntiles = (Q + 15) >> 4;
  epi.init();
  for (int blk = blockIdx.x; blk * NT < ntiles; blk += gridDim.x) {
    // this lane's pixel in each of the block's tiles (clamped; masked at the end)
    const float2* el[NT];
    const float2* em[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int pix = min(16 * (blk * NT + t) + c16, Q - 1);
      const int im = pix / nl, il = pix - im * nl;
      el[t] = tab.El + (size_t)q * nl + il;
      em[t] = tab.Em + (size_t)q * nm + im;
    }
    v4f acc[RPW][NT];
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[i][t] = v4f{0.f, 0.f, 0.f, 0.f};
    const float* fw = frag + (size_t)w * KS * 64 + lane;  // row tile w, chunk 0
    const size_t rstep = (size_t)4 * KS * 64;             // next row tile of this wave
    if constexpr (kPrefetch) {
      float2 te[NT], tm[NT];
      float f0[RPW], f1[RPW];
  #pragma unroll
      for (int t = 0; t < NT; ++t) {
        te[t] = el[t][0];
        tm[t] = em[t][0];
      }
  #pragma unroll
      for (int i = 0; i < RPW; ++i) {
        f0[i] = fw[i * rstep];
        f1[i] = fw[i * rstep + 64];
      }
      for (int j = 0; j < KS / 2; ++j) {                    // chunk pair 2j, 2j + 1: antenna 4j + q
        float b0[NT], b1[NT];
  #pragma unroll
        for (int t = 0; t < NT; ++t) {
          const float2 a = cmul(te[t], tm[t]);
          b0[t] = a.x;
          b1[t] = a.y;
        }
        float g0[RPW], g1[RPW];
  #pragma unroll
        for (int i = 0; i < RPW; ++i) {
          g0[i] = f0[i];
          g1[i] = f1[i];
        }
        const int jn = j + 1 < KS / 2 ? j + 1 : j;  // loads of the next pair
  #pragma unroll
        for (int t = 0; t < NT; ++t) {
          te[t] = el[t][(size_t)4 * jn * nl];
          tm[t] = em[t][(size_t)4 * jn * nm];
        }
  #pragma unroll
        for (int i = 0; i < RPW; ++i) {
          f0[i] = fw[i * rstep + (size_t)(2 * jn) * 64];
          f1[i] = fw[i * rstep + (size_t)(2 * jn + 1) * 64];
        }
  #pragma unroll
        for (int i = 0; i < RPW; ++i)
  #pragma unroll
          for (int t = 0; t < NT; ++t) {
            acc[i][t] = mfma16x16x4(g0[i], b0[t], acc[i][t]);
            acc[i][t] = mfma16x16x4(g1[i], b1[t], acc[i][t]);
          }
      }
    } else {
      for (int j = 0; j < KS / 2; ++j) {                    // chunk pair 2j, 2j + 1: antenna 4j + q
        float b0[NT], b1[NT];
  #pragma unroll
        for (int t = 0; t < NT; ++t) {
          const float2 a = cmul(el[t][(size_t)4 * j * nl], em[t][(size_t)4 * j * nm]);
          b0[t] = a.x;
          b1[t] = a.y;
        }
        float f0[RPW], f1[RPW];
  #pragma unroll
        for (int i = 0; i < RPW; ++i) {
          f0[i] = fw[i * rstep + (size_t)(2 * j) * 64];
          f1[i] = fw[i * rstep + (size_t)(2 * j + 1) * 64];
        }
  #pragma unroll
        for (int i = 0; i < RPW; ++i)
  #pragma unroll
          for (int t = 0; t < NT; ++t) {
            acc[i][t] = mfma16x16x4(f0[i], b0[t], acc[i][t]);
            acc[i][t] = mfma16x16x4(f1[i], b1[t], acc[i][t]);
          }
      }
    }
    // column dot over this wave's row tiles: accumulator element r of row tile m
    // pairs with chunk 4m + r, i.e. antenna 8m + 4(r >> 1) + q, component r & 1
    float gp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      gp[t] = 0.f;
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        const int m = w + 4 * i;
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

bool beam_fits(int P) { return pad_p(P) / 8 <= kBeamMaxMT; }

constexpr int kBigMaxRPW = 9;  // up to 36 row tiles: P <= 288
bool beam_big_fits(int P) { return big_rpw(pad_p(P) / 8) <= kBigMaxRPW; }

size_t beam_big_frag_floats(int P) {
  const int MT = pad_p(P) / 8;
  return (size_t)4 * big_rpw(MT) * 4 * MT * 64;
}

int beam_big_grid(int P, int Q) {
  const int nt = big_nt(big_rpw(pad_p(P) / 8));
  const int nblk = ((Q + 15) / 16 + nt - 1) / nt;
  return nblk < 1 ? 1 : (nblk > 8192 ? 8192 : nblk);
}

int beam_grid(int Q) {
  const int ntiles = (Q + 15) / 16;
  int g = (ntiles + kBeamWaves - 1) / kBeamWaves;
  return g < 1 ? 1 : (g > 2048 ? 2048 : g);
}

hipError_t launch_beam_prep(const float2* U, int P, float* frag, hipStream_t st) {
  const int MT = pad_p(P) / 8;
  const int n = 2 * MT * (MT + 1) * 64;
  hipLaunchKernelGGL(beam_prep_kernel, dim3((n + 255) / 256), dim3(256), 0, st, U, P, MT, frag);
  return hipGetLastError();
}

template <class Epi>
static hipError_t launch_beam(const float* frag, const float2* U, int P, const Tables& tab, const int* skip,
                              Epi epi, hipStream_t st) {
  const dim3 g(beam_grid(tab.Q)), b(64 * kBeamWaves);
  switch (tab.Pp / 8) {
    case 1: hipLaunchKernelGGL((beam_kernel<1, Epi>), g, b, 0, st, frag, U, P, tab, skip, epi); break;
    case 2: hipLaunchKernelGGL((beam_kernel<2, Epi>), g, b, 0, st, frag, U, P, tab, skip, epi); break;
    case 3: hipLaunchKernelGGL((beam_kernel<3, Epi>), g, b, 0, st, frag, U, P, tab, skip, epi); break;
    case 4: hipLaunchKernelGGL((beam_kernel<4, Epi>), g, b, 0, st, frag, U, P, tab, skip, epi); break;
    case 5: hipLaunchKernelGGL((beam_kernel<5, Epi>), g, b, 0, st, frag, U, P, tab, skip, epi); break;
    case 6: hipLaunchKernelGGL((beam_kernel<6, Epi>), g, b, 0, st, frag, U, P, tab, skip, epi); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_beam_prep_full(const float2* U, int P, float* frag, hipStream_t st) {
  const int MT = pad_p(P) / 8;
  const size_t n = beam_big_frag_floats(P);
  int g = (int)((n + 255) / 256);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(beam_prep_full_kernel, dim3(g), dim3(256), 0, st, U, P, MT, frag);
  return hipGetLastError();
}

template <class Epi>
static hipError_t launch_big(const float* frag, const Tables& tab, const int* skip, Epi epi, hipStream_t st) {
  const int MT = tab.Pp / 8;
  const dim3 g(beam_big_grid(tab.Pp, tab.Q)), b(256);
  switch (big_rpw(MT)) {
    case 1: hipLaunchKernelGGL((beam_big_kernel<1, Epi>), g, b, 0, st, frag, MT, tab, skip, epi); break;
    case 2: hipLaunchKernelGGL((beam_big_kernel<2, Epi>), g, b, 0, st, frag, MT, tab, skip, epi); break;
    case 3: hipLaunchKernelGGL((beam_big_kernel<3, Epi>), g, b, 0, st, frag, MT, tab, skip, epi); break;
    case 4: hipLaunchKernelGGL((beam_big_kernel<4, Epi>), g, b, 0, st, frag, MT, tab, skip, epi); break;
    case 5: hipLaunchKernelGGL((beam_big_kernel<5, Epi>), g, b, 0, st, frag, MT, tab, skip, epi); break;
    case 6: hipLaunchKernelGGL((beam_big_kernel<6, Epi>), g, b, 0, st, frag, MT, tab, skip, epi); break;
    case 7: hipLaunchKernelGGL((beam_big_kernel<7, Epi>), g, b, 0, st, frag, MT, tab, skip, epi); break;
    case 8: hipLaunchKernelGGL((beam_big_kernel<8, Epi>), g, b, 0, st, frag, MT, tab, skip, epi); break;
    case 9: hipLaunchKernelGGL((beam_big_kernel<9, Epi>), g, b, 0, st, frag, MT, tab, skip, epi); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_beam_big(int kind, const float* frag, const Tables& tab, const int* skip, float* out, float* eps,
                           float eps_scale, double C, double kb, float scale, const uint8_t* state, uint64_t* part,
                           hipStream_t st) {
  switch (kind) {
    case 0: return launch_big(frag, tab, skip, BeamMF{out, eps, eps_scale}, st);
    case 1: return launch_big(frag, tab, skip, BeamMVDR{out, C, kb}, st);
    case 2: return launch_big(frag, tab, skip, BeamStore{out, scale}, st);
    default: return launch_big(frag, tab, skip, BeamLambda{state, part, nullptr, 0}, st);
  }
}

hipError_t launch_beam_mf(const float* frag, const float2* U, int P, const Tables& tab, float* mf, float* eps,
                          float eps_scale, hipStream_t st) {
  return launch_beam(frag, U, P, tab, nullptr, BeamMF{mf, eps, eps_scale}, st);
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

hipError_t launch_beam_lambda(const float* frag, const float2* U, int P, const Tables& tab, const int* skip,
                              const uint8_t* state, uint64_t* part, const float* scale, hipStream_t st) {
  return launch_beam(frag, U, P, tab, skip, BeamLambda{state, part, scale, 0}, st);
}

}  // namespace clsimg
