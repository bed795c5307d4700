// Control kernels of the active-set solve: free/upper set compaction, the
// LSQR scalar recurrences in FP64, the feasibility test and bounded step of
// Table I, and the final argmin of the Lagrange multipliers.
#include "kernels.h"

namespace clsimg {

constexpr int kCtl = 1024;  // single-workgroup control kernels

// ---------------------------------------------------------------------------
// Sorted index lists of F (state 1) and U (state 2); one workgroup.  The
// state array is taken in rounds of 64 KiB: thread t holds the 64 states of
// bytes 64t .. 64t + 63 of the round (four coalesced 16-byte loads, issued
// one round ahead), the counts are scanned with wave shuffles plus one
// exchange of the wave totals, and each thread writes its pixels in order.
// Two barriers per round.
__global__ __launch_bounds__(kCtl) void compact_kernel(const uint8_t* __restrict__ state, int Q,
                                                       int* __restrict__ Flist,
                                                       int* __restrict__ Ulist,
                                                       SolveDecision* dec) {
  constexpr int NW = kCtl / 64, PER = 64, NV = PER / 16;
  __shared__ int wf[NW], wu[NW];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const bool vec = (reinterpret_cast<uintptr_t>(state) & 15) == 0;
  // this thread's states of the round starting at r0; states past Q read as 0 (L)
  auto fetch = [&](int r0, uint4* d) {
    const int i0 = r0 + PER * tid;
    if (vec && i0 + PER <= Q) {
#pragma unroll
      for (int j = 0; j < NV; ++j) d[j] = reinterpret_cast<const uint4*>(state + i0)[j];
    } else {
      uint32_t ws[PER / 4] = {};
      for (int k = 0; k < PER && i0 + k < Q; ++k) ws[k >> 2] |= (uint32_t)state[i0 + k] << (8 * (k & 3));
#pragma unroll
      for (int j = 0; j < NV; ++j) d[j] = make_uint4(ws[4 * j], ws[4 * j + 1], ws[4 * j + 2], ws[4 * j + 3]);
    }
  };
  auto byte_of = [](const uint4* v, int k) -> uint32_t {
    const uint4 q = v[k >> 4];
    const int wd = (k >> 2) & 3;
    const uint32_t x = wd == 0 ? q.x : wd == 1 ? q.y : wd == 2 ? q.z : q.w;
    return (x >> (8 * (k & 3))) & 0xFFu;
  };
  int baseF = 0, baseU = 0;  // pixels of F and U in the rounds before (the same in every thread)
  uint4 nxt[NV];
  fetch(0, nxt);
  for (int r0 = 0; r0 < Q; r0 += PER * kCtl) {
    uint4 cur[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) cur[j] = nxt[j];
    if (r0 + PER * kCtl < Q) fetch(r0 + PER * kCtl, nxt);
    const int i0 = r0 + PER * tid;
    // states are 0, 1 or 2: byte b is 1 when its bit 0 is set and bit 1
    // clear, 2 when bit 1 is set and bit 0 clear (four bytes per popcount)
    int cf = 0, cu = 0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const uint32_t x[4] = {cur[j].x, cur[j].y, cur[j].z, cur[j].w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cf += __popc(x[q] & ~(x[q] >> 1) & 0x01010101u);
        cu += __popc((x[q] >> 1) & ~x[q] & 0x01010101u);
      }
    }
    int sf = cf, su = cu;  // inclusive scan over the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int tf = __shfl_up(sf, o, 64), tu = __shfl_up(su, o, 64);
      if (lane >= o) {
        sf += tf;
        su += tu;
      }
    }
    if (lane == 63) {
      wf[w] = sf;
      wu[w] = su;
    }
    __syncthreads();
    int pf = 0, pu = 0, tf = 0, tu = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      if (k < w) {
        pf += wf[k];
        pu += wu[k];
      }
      tf += wf[k];
      tu += wu[k];
    }
    int of = baseF + pf + sf - cf, ou = baseU + pu + su - cu;
    if (cf + cu > 0) {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const uint32_t sv = byte_of(cur, k);
        if (sv == 1) Flist[of++] = i0 + k;
        else if (sv == 2) Ulist[ou++] = i0 + k;
      }
    }
    baseF += tf;
    baseU += tu;
    __syncthreads();  // the wave totals are rewritten in the next round
  }
  if (tid == 0) {
    dec->nF = baseF;
    dec->nU = baseU;
  }
}

// ---------------------------------------------------------------------------
// LSQR start: beta_1 = ||b||, alpha_1 = ||M^H u_1||, v_1, w_1 = v_1, x = 0.
__global__ __launch_bounds__(kCtl) void lsqr_init_kernel(LsqrState* s, const double* beta_part,
                                                         int nbeta, const double* alpha_part,
                                                         int nalpha, float* v, float* w, float* x,
                                                         int n, double atol, double btol,
                                                         double conlim, int itnlim) {
  __shared__ double sab[2];
  if (threadIdx.x < 64) {  // wave 0: the norm partials in a fixed order
    const double a2 = wave_sum_parts(alpha_part, nalpha), b2 = wave_sum_parts(beta_part, nbeta);
    if (threadIdx.x == 0) {
      sab[0] = sqrt(a2);
      sab[1] = sqrt(b2);
    }
  }
  __syncthreads();
  const double alpha = sab[0], beta = sab[1];
  const double ia = alpha > 0.0 ? 1.0 / alpha : 0.0;
  for (int k = threadIdx.x; k < n; k += kCtl) {
    const float vk = (float)((double)v[k] * ia);
    v[k] = vk;
    w[k] = vk;
    x[k] = 0.f;
  }
  if (threadIdx.x == 0) {
    s->alpha = alpha;
    s->beta = beta;
    s->rhobar = alpha;
    s->phibar = beta;
    s->bnorm = beta;
    s->anorm2 = 0.0;
    s->ddnorm = 0.0;
    s->rnorm = beta;
    s->arnorm = alpha * beta;
    s->anorm = 0.0;
    s->acond = 0.0;
    s->xnorm = 0.0;
    s->atol = atol;
    s->btol = btol;
    s->conlim = conlim;
    s->itn = 0;
    s->itnlim = itnlim;
    const bool stop = (n == 0) || (beta == 0.0) || (alpha == 0.0);
    s->istop = stop ? 4 : 0;
    s->done = stop ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// One LSQR update after the bidiagonalisation step has produced beta_{i+1}
// (partials of ||u||^2) and the unnormalised v (partials of ||v||^2).
__global__ __launch_bounds__(kCtl) void lsqr_update_kernel(LsqrState* s, const double* beta_part,
                                                           int nbeta, const double* alpha_part,
                                                           int nalpha, float* v, float* w,
                                                           float* x, int n) {
  __shared__ double sc[8];
  __shared__ double red_d[kCtl / 64], red_x[kCtl / 64];
  if (s->done) return;
  double b2 = 0.0, a2 = 0.0;
  if (threadIdx.x < 64) {  // wave 0: the norm partials in a fixed order
    b2 = wave_sum_parts(beta_part, nbeta);
    a2 = wave_sum_parts(alpha_part, nalpha);
  }
  if (threadIdx.x == 0) lsqr_scalars(s, b2, a2, sc);
  __syncthreads();
  double dd = 0.0, xx = 0.0;
  for (int k = threadIdx.x; k < n; k += kCtl) lsqr_vectors(sc, v[k], w[k], x[k], v, w, x, k, dd, xx);
  dd = block_sum_dpp_d(dd, red_d);
  xx = block_sum_dpp_d(xx, red_x);
  if (threadIdx.x == 0) lsqr_close(s, dd, xx, sc[4]);
}

// ---------------------------------------------------------------------------
// Table I, after the subproblem: accept z if 0 <= z <= gamma on F, otherwise
// move along p = z - sigma_F by the largest feasible step (eq. mumax) and move
// the first blocking pixel to its bound.  Sets dec->grad_done = 0 only when a
// feasible z was accepted (the gradient kernels run only then).
__global__ __launch_bounds__(kCtl) void step_kernel(const int* done, const int* err, const LsqrState* s,
                                                    const float* __restrict__ x0,
                                                    const float* __restrict__ x1,
                                                    const int* __restrict__ Flist, int nF,
                                                    float* __restrict__ sigma,
                                                    const float* __restrict__ gamma,
                                                    uint8_t* __restrict__ state,
                                                    SolveDecision* dec) {
  __shared__ int s_ok[kCtl / 64];
  __shared__ double s_mu[kCtl / 64];
  __shared__ int s_k[kCtl / 64];
  __shared__ float s_mz[kCtl / 64];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  // the flags, the iteration count and this thread's first list entry with
  // both iterate buffers are requested together, then its bound
  const int fin = nF > 0 ? *done : 1;
  const int itn = nF > 0 ? s->itn : 0;
  int f0 = 0;
  float z0a = 0.f, z0b = 0.f;
  if (tid < nF) {
    f0 = Flist[tid];
    z0a = x0[tid];
    z0b = x1[tid];
  }
  if (!fin) {
    if (tid == 0) {
      dec->lsqr_done = 0;
      dec->grad_done = 1;
      dec->lsqr_err = err ? *err : 0;
    }
    return;
  }
  const float g0 = tid < nF ? gamma[f0] : 0.f;
  // the final LSQR iterate x_itn is kept in buffer itn & 1
  const float* __restrict__ x = (itn & 1) ? x1 : x0;
  // feasibility (non-strict, no tolerance)
  int ok = 1;
  float mz = 3.0e38f;
  for (int k = tid; k < nF; k += kCtl) {
    const bool pre = k == tid;
    const float z = pre ? ((itn & 1) ? z0b : z0a) : x[k], g = pre ? g0 : gamma[Flist[k]];
    ok &= (z >= 0.f) && (z <= g);
    mz = fminf(mz, fminf(z, g - z) / g);
  }
  for (int o = 32; o > 0; o >>= 1) {
    ok &= __shfl_xor(ok, o, 64);
    mz = fminf(mz, __shfl_xor(mz, o, 64));
  }
  if (lane == 0) {
    s_ok[wv] = ok;
    s_mz[wv] = mz;
  }
  __syncthreads();
  ok = 1;
  mz = 3.0e38f;
  for (int i = 0; i < kCtl / 64; ++i) {
    ok &= s_ok[i];
    mz = fminf(mz, s_mz[i]);
  }
  if (ok) {
    for (int k = tid; k < nF; k += kCtl) sigma[Flist[k]] = x[k];
    if (tid == 0) {
      dec->lsqr_done = 1;
      dec->lsqr_itn = itn;
      dec->lsqr_istop = nF > 0 ? s->istop : 0;
      dec->feasible = 1;
      dec->lsqr_err = 0;
      dec->margin_z = mz;
      dec->ib = -1;
      dec->grad_done = 0;
    }
    return;
  }
  // largest feasible step; ties to the lowest list position (= lowest pixel)
  double best = INFINITY;
  int bk = 0x7fffffff;
  for (int k = tid; k < nF; k += kCtl) {
    const int i = Flist[k];
    const double sg = sigma[i], p = (double)x[k] - sg;
    if (p != 0.0) {
      const double mu = fmax(-sg / p, ((double)gamma[i] - sg) / p);
      if (mu < best || (mu == best && k < bk)) {
        best = mu;
        bk = k;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int ok2 = __shfl_xor(bk, o, 64);
    if (ob < best || (ob == best && ok2 < bk)) {
      best = ob;
      bk = ok2;
    }
  }
  if (lane == 0) {
    s_mu[wv] = best;
    s_k[wv] = bk;
  }
  __syncthreads();
  best = INFINITY;
  bk = 0x7fffffff;
  for (int i = 0; i < kCtl / 64; ++i) {
    if (s_mu[i] < best || (s_mu[i] == best && s_k[i] < bk)) {
      best = s_mu[i];
      bk = s_k[i];
    }
  }
  if (bk >= nF) {  // no finite step (non-finite z): stop moving, block the first pixel
    bk = 0;
    best = 0.0;
  }
  const double mu = best;
  // sign of the step at the blocking pixel, read before any sigma changes
  __shared__ double s_pb;
  if (tid == 0) s_pb = (double)x[bk] - (double)sigma[Flist[bk]];
  __syncthreads();
  // every list entry is owned by one thread: read-modify-write is race free
  for (int k = tid; k < nF; k += kCtl) {
    const int i = Flist[k];
    const double sg = sigma[i], p = (double)x[k] - sg;
    sigma[i] = (float)fmin(fmax(sg + mu * p, 0.0), (double)gamma[i]);
  }
  __syncthreads();
  if (tid == 0) {
    const int ib = Flist[bk];
    const bool to_upper = !(s_pb < 0.0);
    sigma[ib] = to_upper ? gamma[ib] : 0.f;
    state[ib] = to_upper ? (uint8_t)2 : (uint8_t)0;
    dec->lsqr_done = 1;
    dec->lsqr_itn = s->itn;
    dec->lsqr_istop = s->istop;
    dec->feasible = 0;
    dec->lsqr_err = 0;
    dec->ib = ib;
    dec->ib_to = to_upper ? 2 : 0;
    dec->mu_max = (float)mu;
    dec->grad_done = 1;
  }
}

// ---------------------------------------------------------------------------
// cand_count / cand_cap (optional): the refined multipliers' candidate list;
// if it overflowed, the decision is left open (grad_done stays 0,
// cand_overflow = 1) for a full FP32 evaluation.
__global__ __launch_bounds__(kCtl) void argmin_final_kernel(const uint64_t* __restrict__ part,
                                                            int nparts,
                                                            const float* __restrict__ eps,
                                                            const uint8_t* __restrict__ state,
                                                            SolveDecision* dec, const int* cand_count,
                                                            int cand_cap) {
  __shared__ uint64_t sh[kCtl / 64];
  if (dec->grad_done) return;
  if (cand_count) {
    const int over = *cand_count > cand_cap;
    if (threadIdx.x == 0) dec->cand_overflow = over;
    if (over) return;
  }
  uint64_t m = ~0ull;
  for (int i = threadIdx.x; i < nparts; i += kCtl) m = part[i] < m ? part[i] : m;
  m = block_min_u64(m, sh);
  if (threadIdx.x == 0) {
    if (m == ~0ull) {
      dec->i_min = -1;
      dec->lam_min = 0.f;
      dec->eps_min = 0.f;
    } else {
      const int i = (int)(m & 0xffffffffu);
      dec->i_min = i;
      dec->st_min = state[i];
      dec->lam_min = from_ordered_bits((uint32_t)(m >> 32));
      dec->eps_min = eps[i];
    }
    dec->grad_done = 1;
  }
}

__global__ void set_state_kernel(uint8_t* state, int i, uint8_t v) { state[i] = v; }

__global__ void init_state_kernel(const float* __restrict__ sigma0, const uint8_t* __restrict__ state0,
                                  float* __restrict__ sigma, uint8_t* __restrict__ state, int Q) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < Q; e += gridDim.x * blockDim.x) {
    sigma[e] = sigma0 ? sigma0[e] : 0.f;
    const uint8_t v = state0 ? state0[e] : (uint8_t)0;
    state[e] = v <= 2 ? v : (uint8_t)0;  // values other than F and U read as L
  }
}

// ---------------------------------------------------------------------------
// ---- compaction over many workgroups: chunks of kCmpChunk states ----
// compact_count_kernel: the F and U counts of each chunk (part[2b], part[2b+1]);
// compact_write_kernel: each chunk's offsets from the counts of the chunks
// before it, a scan inside the chunk, and its entries of the sorted lists; the
// last chunk writes the totals.
constexpr int kCmpThreads = 256, kCmpChunk = kCmpThreads * 16;

// sixteen states from i0 (past Q: 0, the lower set), as four words
__device__ inline uint4 cmp_load(const uint8_t* __restrict__ state, int Q, int i0, bool vec) {
  if (vec && i0 + 16 <= Q) return *reinterpret_cast<const uint4*>(state + i0);
  uint32_t ws[4] = {0u, 0u, 0u, 0u};
  for (int k = 0; k < 16 && i0 + k < Q; ++k) ws[k >> 2] |= (uint32_t)state[i0 + k] << (8 * (k & 3));
  return make_uint4(ws[0], ws[1], ws[2], ws[3]);
}

// states are 0, 1 or 2: byte b is 1 when its bit 0 is set and bit 1 clear, 2
// when bit 1 is set and bit 0 clear (four bytes per popcount)
__device__ inline void cmp_count(uint4 v, int& cf, int& cu) {
  const uint32_t x[4] = {v.x, v.y, v.z, v.w};
  cf = 0;
  cu = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    cf += __popc(x[q] & ~(x[q] >> 1) & 0x01010101u);
    cu += __popc((x[q] >> 1) & ~x[q] & 0x01010101u);
  }
}

__global__ __launch_bounds__(kCmpThreads) void compact_count_kernel(const uint8_t* __restrict__ state, int Q,
                                                                    int* __restrict__ part) {
  __shared__ int sf[kCmpThreads / 64], su[kCmpThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const bool vec = (reinterpret_cast<uintptr_t>(state) & 15) == 0;
  int cf, cu;
  cmp_count(cmp_load(state, Q, blockIdx.x * kCmpChunk + 16 * tid, vec), cf, cu);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    cf += __shfl_xor(cf, o, 64);
    cu += __shfl_xor(cu, o, 64);
  }
  if (lane == 0) {
    sf[w] = cf;
    su[w] = cu;
  }
  __syncthreads();
  if (tid == 0) {
    int tf = 0, tu = 0;
#pragma unroll
    for (int k = 0; k < kCmpThreads / 64; ++k) {
      tf += sf[k];
      tu += su[k];
    }
    part[2 * blockIdx.x] = tf;
    part[2 * blockIdx.x + 1] = tu;
  }
}

__global__ __launch_bounds__(kCmpThreads) void compact_write_kernel(const uint8_t* __restrict__ state, int Q,
                                                                    const int* __restrict__ part,
                                                                    int* __restrict__ Flist, int* __restrict__ Ulist,
                                                                    SolveDecision* dec) {
  constexpr int NW = kCmpThreads / 64;
  __shared__ int wf[NW], wu[NW], base[2];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, b = blockIdx.x;
  const bool vec = (reinterpret_cast<uintptr_t>(state) & 15) == 0;
  const int i0 = b * kCmpChunk + 16 * tid;
  const uint4 v = cmp_load(state, Q, i0, vec);
  if (w == 0) {  // the chunks before this one
    int pf = 0, pu = 0;
    for (int k = lane; k < b; k += 64) {
      pf += part[2 * k];
      pu += part[2 * k + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      pf += __shfl_xor(pf, o, 64);
      pu += __shfl_xor(pu, o, 64);
    }
    if (lane == 0) {
      base[0] = pf;
      base[1] = pu;
    }
  }
  int cf, cu;
  cmp_count(v, cf, cu);
  int sf = cf, su = cu;  // inclusive scan over the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int tf = __shfl_up(sf, o, 64), tu = __shfl_up(su, o, 64);
    if (lane >= o) {
      sf += tf;
      su += tu;
    }
  }
  if (lane == 63) {
    wf[w] = sf;
    wu[w] = su;
  }
  __syncthreads();
  int pf = base[0], pu = base[1], tf = 0, tu = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    if (k < w) {
      pf += wf[k];
      pu += wu[k];
    }
    tf += wf[k];
    tu += wu[k];
  }
  int of = pf + sf - cf, ou = pu + su - cu;
  if (cf + cu > 0) {
    const uint32_t x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t sv = (x[k >> 2] >> (8 * (k & 3))) & 0xFFu;
      if (sv == 1) Flist[of++] = i0 + k;
      else if (sv == 2) Ulist[ou++] = i0 + k;
    }
  }
  if (b == gridDim.x - 1 && tid == 0) {
    dec->nF = base[0] + tf;
    dec->nU = base[1] + tu;
  }
}

int compact_parts(int Q) { return 2 * ((Q + kCmpChunk - 1) / kCmpChunk); }

hipError_t launch_compact(const uint8_t* state, int Q, int* Flist, int* Ulist, SolveDecision* dec, int* part,
                          hipStream_t st) {
  if (Q <= 0) return hipErrorInvalidValue;
  const int nb = (Q + kCmpChunk - 1) / kCmpChunk;
  if (nb == 1) {
    hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(kCtl), 0, st, state, Q, Flist, Ulist, dec);
  } else {
    hipLaunchKernelGGL(compact_count_kernel, dim3(nb), dim3(kCmpThreads), 0, st, state, Q, part);
    hipLaunchKernelGGL(compact_write_kernel, dim3(nb), dim3(kCmpThreads), 0, st, state, Q, (const int*)part, Flist,
                       Ulist, dec);
  }
  return hipGetLastError();
}

hipError_t launch_lsqr_init_scalars(LsqrState* s, const double* beta_part, int nbeta,
                                    const double* alpha_part, int nalpha, float* v, float* w,
                                    float* x, int n, double atol, double btol, double conlim,
                                    int itnlim, hipStream_t st) {
  hipLaunchKernelGGL(lsqr_init_kernel, dim3(1), dim3(kCtl), 0, st, s, beta_part, nbeta, alpha_part,
                     nalpha, v, w, x, n, atol, btol, conlim, itnlim);
  return hipGetLastError();
}

// LSQR over K covariance blocks: v <- (sum_k g_k) / beta - beta v (or the sum
// / beta at the start), the block dots g_k = gpart[k * stride + col] added in
// block order; one 64-column tile per workgroup, its sum of v^2 to
// alpha_part[tile] (the tiles of the adjoint's own LSQR epilogue).
__global__ __launch_bounds__(64) void lsqr_v_blocks_kernel(const float* __restrict__ gpart, int K, size_t stride,
                                                           int n, float* __restrict__ v,
                                                           const double* __restrict__ beta_part, int nbeta,
                                                           double* __restrict__ alpha_part, int first,
                                                           const int* stop) {
  if (stop && *stop) return;
  const int col = blockIdx.x * 64 + threadIdx.x;
  const double beta = sqrt(wave_sum_parts(beta_part, nbeta));
  double vr2 = 0.0;
  if (col < n) {
    float g = 0.f;
    for (int k = 0; k < K; ++k) g += gpart[k * stride + col];
    double vr = beta > 0.0 ? (double)g / beta : 0.0;
    if (!first) vr -= beta * (double)v[col];
    const float vf = (float)vr;
    v[col] = vf;
    vr2 = (double)vf * vf;
  }
  vr2 = wave_sum_d(vr2);
  if (threadIdx.x == 0) alpha_part[blockIdx.x] = vr2;
}

hipError_t launch_lsqr_v_blocks(const float* gpart, int K, size_t stride, int n, float* v, const double* beta_part,
                                int nbeta, double* alpha_part, int first, const int* stop, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lsqr_v_blocks_kernel, dim3((n + 63) / 64), dim3(64), 0, st, gpart, K, stride, n, v, beta_part,
                     nbeta, alpha_part, first, stop);
  return hipGetLastError();
}

hipError_t launch_lsqr_update(LsqrState* s, const double* beta_part, int nbeta,
                              const double* alpha_part, int nalpha, float* v, float* w, float* x,
                              int n, hipStream_t st) {
  hipLaunchKernelGGL(lsqr_update_kernel, dim3(1), dim3(kCtl), 0, st, s, beta_part, nbeta,
                     alpha_part, nalpha, v, w, x, n);
  return hipGetLastError();
}

hipError_t launch_step(const int* done, const int* err, const LsqrState* s, const float* x0,
                       const float* x1, const int* Flist, int nF, float* sigma, const float* gamma,
                       uint8_t* state, SolveDecision* dec, hipStream_t st) {
  hipLaunchKernelGGL(step_kernel, dim3(1), dim3(kCtl), 0, st, done, err, s, x0, x1, Flist, nF, sigma,
                     gamma, state, dec);
  return hipGetLastError();
}

hipError_t launch_argmin_final(const uint64_t* part, int nparts, const float* eps,
                               const uint8_t* state, SolveDecision* dec, hipStream_t st, const int* cand_count, int cand_cap) {
  hipLaunchKernelGGL(argmin_final_kernel, dim3(1), dim3(kCtl), 0, st, part, nparts, eps, state, dec, cand_count,
                     cand_cap);
  return hipGetLastError();
}

hipError_t launch_set_state(uint8_t* state, int i, uint8_t v, hipStream_t st) {
  hipLaunchKernelGGL(set_state_kernel, dim3(1), dim3(1), 0, st, state, i, v);
  return hipGetLastError();
}

hipError_t launch_init_state(const float* sigma0, const uint8_t* state0, float* sigma,
                             uint8_t* state, int Q, hipStream_t st) {
  int grid = (Q + 255) / 256;
  if (grid > 2048) grid = 2048;
  hipLaunchKernelGGL(init_state_kernel, dim3(grid), dim3(256), 0, st, sigma0, state0, sigma, state,
                     Q);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K covariance blocks (eq. vectRtotal).  The full-grid beamformer leaves the
// block sums; these kernels turn them into the threshold, the bound and the
// multiplier keys.
//   MF:   mf = (1/K) sum_k m_k (summed by the beamformer), eps = kappa_d
//         sqrt(sum_k m_k^2) / (K sqrt N)                       (App. A)
//   MVDR: gamma = C K / sum_k h_k + kappa_b K sqrt(sum_k h_k^2) /
//         (sqrt(N - p - 1) (sum_k h_k)^2)                 (eq. wmvdr, App. A)
//   MF bound: gamma = mf + kappa_b sqrt(sum_k m_k^2) / (K sqrt N)
__global__ void multi_mf_kernel(const float* __restrict__ mfsq, int Q, float eps_coef, float* __restrict__ eps) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < Q; i += gridDim.x * blockDim.x)
    eps[i] = eps_coef * sqrtf(mfsq[i]);
}

__global__ void multi_bound_kernel(int kind, const float* __restrict__ s1, const float* __restrict__ s2, int Q,
                                   double C, double K, double kb_coef, float* __restrict__ gamma) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < Q; i += gridDim.x * blockDim.x) {
    const double a = s1[i], b = s2[i];
    double g;
    if (kind == 0) {  // MVDR from the sums of h_k and h_k^2
      g = C * K / a;
      if (kb_coef != 0.0) g += kb_coef * K * sqrt(b) / (a * a);
    } else {  // MF from the image and the sum of m_k^2
      g = a + kb_coef * sqrt(b);
    }
    gamma[i] = (float)g;
  }
}

// keys (ordered lambda << 32 | pixel) of the active pixels from a gradient
// vector: lambda = g on L, -g on U; one key per block
__global__ __launch_bounds__(256) void lambda_vec_kernel(const float* __restrict__ g,
                                                         const uint8_t* __restrict__ state, int Q,
                                                         const int* skip, uint64_t* __restrict__ part) {
  __shared__ uint64_t sh[4];
  if (skip && *skip) return;
  uint64_t best = ~0ull;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < Q; i += gridDim.x * blockDim.x) {
    const uint8_t s = state[i];
    if (s == 1) continue;
    const float lam = s == 0 ? g[i] : -g[i];
    const uint64_t key = ((uint64_t)ordered_bits(lam) << 32) | (uint32_t)i;
    best = key < best ? key : best;
  }
  best = block_min_u64(best, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = best;
}

hipError_t launch_multi_mf(const float* mfsq, int Q, float eps_coef, float* eps, hipStream_t st) {
  const int g = std::min((Q + 255) / 256, 2048);
  hipLaunchKernelGGL(multi_mf_kernel, dim3(g), dim3(256), 0, st, mfsq, Q, eps_coef, eps);
  return hipGetLastError();
}

hipError_t launch_multi_bound(int kind, const float* s1, const float* s2, int Q, double C, double K, double kb_coef,
                              float* gamma, hipStream_t st) {
  const int g = std::min((Q + 255) / 256, 2048);
  hipLaunchKernelGGL(multi_bound_kernel, dim3(g), dim3(256), 0, st, kind, s1, s2, Q, C, K, kb_coef, gamma);
  return hipGetLastError();
}

int lambda_vec_blocks(int Q) { return std::max(1, std::min((Q + 255) / 256, 1024)); }

hipError_t launch_lambda_vec(const float* g, const uint8_t* state, int Q, const int* skip, uint64_t* part,
                             hipStream_t st) {
  hipLaunchKernelGGL(lambda_vec_kernel, dim3(lambda_vec_blocks(Q)), dim3(256), 0, st, g, state, Q, skip, part);
  return hipGetLastError();
}

}  // namespace clsimg
