// Internal device/host helpers of the clsimg HIP library (gfx950 only).
//
// Data layout used by every kernel
// --------------------------------
//  * P is padded to Pp = ceil(P/8)*8.  Padding antennas have a zero response.
//  * Complex steering vectors are handled in an interleaved real embedding:
//    x_i = [Re a_i[0], Im a_i[0], Re a_i[1], Im a_i[1], ...]  (length 2Pp).
//    For a Hermitian U, Re(a^H U a) = x^T Ut x with the real 2Pp x 2Pp matrix
//        Ut[2p+s][2q+t] = { Re U_pq  (s,t)=(0,0),(1,1);  -Im U_pq (0,1);  Im U_pq (1,0) }
//    and sum_i v_i a_i a_i^H is assembled from G = X diag(v) X^T as
//        Re = G[2p][2q] + G[2p+1][2q+1],  Im = G[2p+1][2q] - G[2p][2q+1].
//    Both products are plain real GEMMs with M = N or K = 2Pp (a multiple of
//    16), which run on the fp32 MFMA v_mfma_f32_16x16x4f32.
//  * Steering tables (complex64, built in FP64 on the host):
//        El[p*nl + il] = P^-1/2 exp(-j 2pi x_p l_il / lambda)
//        Em[p*nm + im] =        exp(-j 2pi y_p m_im / lambda)
//    so a_i[p] = El[p][il] * Em[p][im] for pixel i = im*nl + il: one complex
//    multiply per entry, no transcendental in any kernel, ~1 ulp of fp32.
//  * MFMA 16x16x4 f32 lane layout (lane l, c16 = l%16, q = l/16):
//        A operand: A[c16][q];  B operand: B[q][c16];
//        D (4 regs r): D[4q + r][c16].
//  * "Fragment" order of Ut for the beamforming product Y = Ut X:
//        frag[(mt*KS + kc)*64 + l] = Ut[16 mt + c16][4 kc + q],
//    MT = 2Pp/16 row tiles, KS = 2Pp/4 k-steps, so each MFMA A operand is
//    one contiguous 256-byte load.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace clsimg {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;  // every multi-wave kernel: 4 waves of 64

__host__ __device__ inline int pad_p(int P) { return (P + 7) & ~7; }

__device__ __forceinline__ v4f mfma16x16x4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Loads through the global address space.  A pointer read from memory (an
// item of a batched launch) is otherwise accessed with flat instructions,
// which also count against the LDS wait counter, so every LDS or cross-lane
// wait would wait for them too.
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_global(const float2* p) {
  const v2f v = *(const __attribute__((address_space(1))) v2f*)p;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ float ld_global(const float* p) { return *(const __attribute__((address_space(1))) float*)p; }
__device__ __forceinline__ int ld_global(const int* p) { return *(const __attribute__((address_space(1))) int*)p; }
__device__ __forceinline__ uint8_t ld_global(const uint8_t* p) {
  return *(const __attribute__((address_space(1))) uint8_t*)p;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Steering-table view shared by the operator kernels.
// Correlation tiling (forward operator): 16-antenna tiles, blocks of BT x BT
// tile pairs, only block pairs on and below the diagonal; corr_rows is the
// antennas a block row covers in all (the row length of the antenna-fastest
// tables).  They depend on Pp only.
__host__ __device__ inline int corr_tiles(int P) { return (pad_p(P) + 15) / 16; }
__host__ __device__ inline int corr_bt(int P) { return corr_tiles(P) <= 2 ? 2 : 3; }
__host__ __device__ inline int corr_nblocks(int P) { return (corr_tiles(P) + corr_bt(P) - 1) / corr_bt(P); }
__host__ __device__ inline int corr_pairs(int P) { return corr_nblocks(P) * (corr_nblocks(P) + 1) / 2; }
__host__ __device__ inline int corr_rows(int P) { return 16 * corr_bt(P) * corr_nblocks(P); }

struct Tables {
  const float2* El;  // Pp x nl
  const float2* Em;  // Pp x nm
  int nl, nm, Pp, Q;
  // the same tables antenna-fastest (nl x corr_rows(Pp), nm x corr_rows(Pp),
  // zero beyond Pp), or null: the correlation reads 16 consecutive antennas
  // of one pixel per lane group
  const float2* ElT = nullptr;
  const float2* EmT = nullptr;
  __device__ __forceinline__ float2 a(int p, int il, int im) const {
    return cmul(El[p * nl + il], Em[p * nm + im]);
  }
};

// Monotone float -> uint32 map so that unsigned comparison orders floats;
// NaN sorts above +inf.
__device__ __forceinline__ uint32_t ordered_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if (f != f) return 0xFFFFFFFFu;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float from_ordered_bits(uint32_t u) {
  uint32_t v = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
  float f;
  __builtin_memcpy(&f, &v, 4);
  return f;
}

// Wave-level (64 lanes) reductions.
__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// DPP move of a double: both 32-bit halves with the same lane pattern; lanes
// whose source is outside the pattern (or whose row is masked off) get 0.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_move_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), kCtrl, kRowMask, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), kCtrl, kRowMask, 0xF, false);
  return __hiloint2double(hi, lo);
}
// Wave sum on the VALU: row_shr 1, 2, 4, 8 leave each 16-lane row's total in
// its lane 15; row_bcast 15 and 31 carry the row totals up to lane 63, which
// every lane then reads.
__device__ __forceinline__ double wave_sum_dpp_d(double v) {
  v += dpp_move_d<0x111, 0xF>(v);
  v += dpp_move_d<0x112, 0xF>(v);
  v += dpp_move_d<0x114, 0xF>(v);
  v += dpp_move_d<0x118, 0xF>(v);
  v += dpp_move_d<0x142, 0xA>(v);
  v += dpp_move_d<0x143, 0xC>(v);
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                          __builtin_amdgcn_readlane(__double2loint(v), 63));
}
// Sum of n doubles by one full wave in a fixed order: lane l adds p[l],
// p[l + 64], ... in turn, then the VALU wave sum (every lane gets lane 63's
// total, so all end with the same bits).  Call with all 64 lanes of a wave.
__device__ inline double wave_sum_parts(const double* p, int n) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int i0 = lane; i0 < n; i0 += 256) {  // four per lane requested before the first add
    double v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = i0 + 64 * j < n ? p[i0 + 64 * j] : 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (i0 + 64 * j < n) s += v[j];
  }
  return wave_sum_dpp_d(s);
}
__device__ __forceinline__ float wave_sum_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}

// Block-level reductions through an LDS scratch of NW slots (one per wave);
// every thread gets the result.  The scratch is passed as an array reference
// so that its size is known: slots beyond NW are never touched.
template <int NW>
__device__ inline double block_sum_d(double v, double (&sh)[NW]) {
  v = wave_sum_d(v);
  const int w = threadIdx.x >> 6;
  const int nw = min((int)(blockDim.x >> 6), NW);
  __syncthreads();
  if ((threadIdx.x & 63) == 0 && w < NW) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += sh[i];
  return s;
}
// block_sum_d with the VALU wave sum (all 64 lanes of every wave active).
template <int NW>
__device__ inline double block_sum_dpp_d(double v, double (&sh)[NW]) {
  v = wave_sum_dpp_d(v);
  const int w = threadIdx.x >> 6;
  const int nw = min((int)(blockDim.x >> 6), NW);
  __syncthreads();
  if ((threadIdx.x & 63) == 0 && w < NW) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += sh[i];
  return s;
}
// Two sums at once through one pair of barriers (NS = 2 slots per wave).
template <int NS>
__device__ inline void block_sum_d2(double& a, double& b, double (&sh)[NS]) {
  constexpr int NW = NS / 2;
  a = wave_sum_d(a);
  b = wave_sum_d(b);
  const int w = threadIdx.x >> 6;
  const int nw = min((int)(blockDim.x >> 6), NW);
  __syncthreads();
  if ((threadIdx.x & 63) == 0 && w < NW) {
    sh[w] = a;
    sh[NW + w] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
  for (int i = 0; i < nw; ++i) {
    sa += sh[i];
    sb += sh[NW + i];
  }
  a = sa;
  b = sb;
}
template <int NW>
__device__ inline uint64_t block_min_u64(uint64_t v, uint64_t (&sh)[NW]) {
  v = wave_min_u64(v);
  const int w = threadIdx.x >> 6;
  const int nw = min((int)(blockDim.x >> 6), NW);
  __syncthreads();
  if ((threadIdx.x & 63) == 0 && w < NW) sh[w] = v;
  __syncthreads();
  uint64_t m = ~0ull;
  for (int i = 0; i < nw; ++i) m = sh[i] < m ? sh[i] : m;
  return m;
}

}  // namespace clsimg
