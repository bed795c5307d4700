// Output-stationary correlation tiles shared by the free-set kernels.
//
// G = X diag(v) X^T is computed one 16 x 16 tile (mt <= nt) per wave; after
// the MFMA the lane (c16, q) holds G[16mt + 4q + r][16nt + c16] (r = 0..3).
// The complex entries are assembled with the neighbouring lane (c16 ^ 1):
//   Re K[p][q] = G[2p][2q] + G[2p+1][2q+1],  Im K[p][q] = G[2p+1][2q] - G[2p][2q+1].
// Lanes with even c16 then own K[p0 + h][qq] (h = 0, 1) and, for an
// off-diagonal tile, the Hermitian mirror K[qq][p0 + h] = conj(K[p0 + h][qq]),
// so every element of the P x P result has exactly one owner.
#pragma once

#include "kernels.h"

namespace clsimg {

// Tile (mt, nt), mt <= nt, of the upper triangle, enumerated row by row.
__device__ inline void tri_tile(int tp, int MT, int& mt, int& nt) {
  int r = tp;
  mt = 0;
  while (r >= MT - mt) {
    r -= MT - mt;
    ++mt;
  }
  nt = mt + r;
}

struct OsSlots {
  int pa[4], pb[4];
  bool live[4], mirror[4];
};

__device__ inline OsSlots os_slots(int mt, int nt, int c16, int q, int P, bool active) {
  OsSlots s;
  const int p0 = 8 * mt + 2 * q, qq = 8 * nt + (c16 >> 1);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int h = i & 1, m = i >> 1;
    s.mirror[i] = m;
    s.pa[i] = m ? qq : p0 + h;
    s.pb[i] = m ? p0 + h : qq;
    s.live[i] = active && (c16 & 1) == 0 && !(m && mt == nt);
  }
  (void)P;
  return s;
}

// Owned elements of B (zero where not owned or padding).
__device__ inline void os_prefetch(const OsSlots& sl, const float2* B, int P, float2* Bold) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    Bold[i] = make_float2(0.f, 0.f);
    if (B && sl.live[i] && sl.pa[i] < P && sl.pb[i] < P) Bold[i] = B[sl.pa[i] * P + sl.pb[i]];
  }
}

// Complex entries of the owned elements from the tile accumulator (all lanes
// must call: it shuffles with the neighbouring lane).
__device__ inline void os_assemble(v4f acc, const OsSlots& sl, float2* K) {
  const float4 s4 = make_float4(acc[0], acc[1], acc[2], acc[3]);
  float4 o4;
  o4.x = __shfl_xor(s4.x, 1, 64);
  o4.y = __shfl_xor(s4.y, 1, 64);
  o4.z = __shfl_xor(s4.z, 1, 64);
  o4.w = __shfl_xor(s4.w, 1, 64);
  const float2 K0 = make_float2(s4.x + o4.y, s4.y - o4.x);
  const float2 K1 = make_float2(s4.z + o4.w, s4.w - o4.z);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float2 k = (i & 1) ? K1 : K0;
    K[i] = sl.mirror[i] ? make_float2(k.x, -k.y) : k;
  }
}

// Store owned values (padding entries as zero) and their Ut fragments;
// returns the sum of |value|^2 over real entries.
__device__ inline double os_store(const OsSlots& sl, const float2* val, int P, int Pp, float2* out,
                                  float* frag) {
  const int KS = Pp / 2;
  double nrm = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (!sl.live[i]) continue;
    const int pa = sl.pa[i], pb = sl.pb[i];
    float2 r = make_float2(0.f, 0.f);
    if (pa < P && pb < P) {
      r = val[i];
      if (out) out[pa * P + pb] = r;
      nrm += (double)r.x * r.x + (double)r.y * r.y;
    }
    if (frag) {
#pragma unroll
      for (int su = 0; su < 4; ++su) {
        const int s_ = su >> 1, u_ = su & 1;
        const int row = 2 * pa + s_, col = 2 * pb + u_;
        const float v = (s_ == u_) ? r.x : (s_ == 0 ? -r.y : r.y);
        frag[((row >> 4) * KS + (col >> 2)) * 64 + (col & 3) * 16 + (row & 15)] = v;
      }
    }
  }
  return nrm;
}

// Tile accumulation over n16 (multiple of 16) LDS-resident pixel rows of
// stride RS with weights w[k]; four independent accumulators.
__device__ inline v4f os_accumulate_lds(const float* xr, const float* w, int n16, int RS, bool active,
                                        int mt, int nt) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, q = lane >> 4;
  v4f acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
  if (active) {
    for (int kk = 0; kk < n16; kk += 16) {
      float a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = kk + 4 * u + q;
        a[u] = xr[k * RS + 16 * mt + c16] * w[k];
        b[u] = xr[k * RS + 16 * nt + c16];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = mfma16x16x4(a[u], b[u], acc[u]);
    }
  }
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

}  // namespace clsimg
