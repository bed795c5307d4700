// Kernel running one single-workgroup LSQR solve on prepared steering vectors.
#include "lsqr_cu.h"

namespace clsimg {

template <int MT>
__global__ __launch_bounds__(kCuThreads) void lsqr_cu_kernel(LsqrCuParams pr) {
  constexpr int Pp = 8 * MT;
  constexpr int RS = cu_row_stride(Pp);
  __shared__ float lds[kCuLds];
  const int tid = threadIdx.x, n = pr.n;
  const int n16 = (n + 15) & ~15;
  for (int e = tid; e < n16 * 2 * Pp; e += kCuThreads) {
    const int k = e / (2 * Pp), r = e - k * (2 * Pp);
    lds[k * RS + r] = k < n ? pr.xf[(size_t)k * 2 * Pp + r] : 0.f;
  }
  __syncthreads();
  const LsqrState S = cu_lsqr<MT>(lds, n, pr.P, pr.B, pr.atol, pr.btol, pr.conlim, pr.itnlim);
  const float* xv = cu_x(lds, MT, n);
  for (int k = tid; k < n; k += kCuThreads) pr.x_out[k] = xv[k];
  __syncthreads();
  if (tid == 0) {
    *pr.Sfinal = S;
    *pr.done = 1;
  }
}

bool lsqr_cu_fits(int P, int n) {
  const int MT = pad_p(P) / 8;
  // up to P = 48 (eight row tiles of the real embedding would not leave room
  // for the steering vectors of a useful free set in LDS)
  return MT <= 6 && n > 0 && cu_lds_floats(MT, n) <= kCuLds;
}

hipError_t launch_lsqr_cu(const LsqrCuParams& pr, hipStream_t st) {
  const dim3 g(1), b(kCuThreads);
  switch (pad_p(pr.P) / 8) {
    case 1: hipLaunchKernelGGL(lsqr_cu_kernel<1>, g, b, 0, st, pr); break;
    case 2: hipLaunchKernelGGL(lsqr_cu_kernel<2>, g, b, 0, st, pr); break;
    case 3: hipLaunchKernelGGL(lsqr_cu_kernel<3>, g, b, 0, st, pr); break;
    case 4: hipLaunchKernelGGL(lsqr_cu_kernel<4>, g, b, 0, st, pr); break;
    case 5: hipLaunchKernelGGL(lsqr_cu_kernel<5>, g, b, 0, st, pr); break;
    case 6: hipLaunchKernelGGL(lsqr_cu_kernel<6>, g, b, 0, st, pr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace clsimg
