// Strong off-grid sources (Sec. III-E, eq. doals): kernels of the offset
// correction of the free pixels.
//
// A free pixel's steering vector is taken at its centre shifted by
// delta_i = (delta_l, delta_m) in direction cosines.  Each subproblem runs
// rounds of (LSQR for sigma_F at the current offsets, one Gauss-Newton step on
// every free pixel's offset with the coupling between pixels neglected); the
// step of pixel i is -(z_i^2 G)^-1 g_i with
//   g_ij = 2 z_i c sum_p x_jp Im(conj(y_p) a_p),  y = E a_i,
//   G    = 2 c^2 Cov(x, y)  (antenna positions averaged over the array),
// c = 2 pi / lambda, E = Psi(delta)_F z - b; it is clipped to half a pixel.
#include "kernels.h"

namespace clsimg {

namespace {

__device__ inline double wave_sum_dbl(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace

// steering vectors of the free list at their shifted directions, the layout
// of xf_kernel (2 Pp floats per pixel: Re, Im per antenna; zero past P); the
// phase is formed in FP64
__global__ void xf_off_kernel(const double* __restrict__ pos, int P, int Pp, double lam, int nl, double l0,
                              double dl, double m0, double dm, const int* __restrict__ Flist, int n,
                              const float* __restrict__ delta, float* __restrict__ xf) {
  const double k2pi = -2.0 * M_PI / lam, rs = 1.0 / sqrt((double)P);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * Pp; e += gridDim.x * blockDim.x) {
    const int k = e / Pp, p = e - k * Pp;
    float2 v = make_float2(0.f, 0.f);
    if (p < P) {
      const int pix = Flist[k];
      const int im = pix / nl, il = pix - im * nl;
      const double l = l0 + il * dl + (double)delta[2 * pix], m = m0 + im * dm + (double)delta[2 * pix + 1];
      double s, c;
      sincos(k2pi * (pos[2 * p] * l + pos[2 * p + 1] * m), &s, &c);
      v = make_float2((float)(c * rs), (float)(s * rs));
    }
    *reinterpret_cast<float2*>(xf + (size_t)k * 2 * Pp + 2 * p) = v;
  }
}

// one wave per free pixel: the Gauss-Newton step of its offset
__global__ __launch_bounds__(256) void newton_offset_kernel(const float2* __restrict__ E, int P, int Pp,
                                                            const double* __restrict__ pos, double lam,
                                                            const int* __restrict__ Flist, int n,
                                                            const float* __restrict__ z,
                                                            const float* __restrict__ xf, float* __restrict__ delta,
                                                            float half_l, float half_m) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (k >= n) return;  // the whole wave
  const float zk = z[k];
  const float* a = xf + (size_t)k * 2 * Pp;
  // y = E a; lane p accumulates rows p, p + 64, ...; sums for the gradient and G
  double g1 = 0.0, g2 = 0.0, sx = 0.0, sy = 0.0, sxx = 0.0, sxy = 0.0, syy = 0.0;
  for (int p = lane; p < P; p += 64) {
    float yr = 0.f, yi = 0.f;
    for (int q = 0; q < P; ++q) {
      const float2 e = E[p * P + q];
      const float ar = a[2 * q], ai = a[2 * q + 1];
      yr += e.x * ar - e.y * ai;
      yi += e.x * ai + e.y * ar;
    }
    const double ar = a[2 * p], ai = a[2 * p + 1];
    const double im = (double)yr * ai - (double)yi * ar;  // Im(conj(y_p) a_p)
    const double x = pos[2 * p], y = pos[2 * p + 1];
    g1 += x * im;
    g2 += y * im;
    sx += x;
    sy += y;
    sxx += x * x;
    sxy += x * y;
    syy += y * y;
  }
  g1 = wave_sum_dbl(g1);
  g2 = wave_sum_dbl(g2);
  sx = wave_sum_dbl(sx);
  sy = wave_sum_dbl(sy);
  sxx = wave_sum_dbl(sxx);
  sxy = wave_sum_dbl(sxy);
  syy = wave_sum_dbl(syy);
  if (lane != 0 || zk == 0.f) return;
  const double c = 2.0 * M_PI / lam, zd = zk;
  const double mx = sx / P, my = sy / P;
  const double f = 2.0 * c * c * zd * zd;  // z^2 G = f Cov
  const double h11 = f * (sxx / P - mx * mx), h12 = f * (sxy / P - mx * my), h22 = f * (syy / P - my * my);
  const double r1 = 2.0 * zd * c * g1, r2 = 2.0 * zd * c * g2;  // gradient
  const double det = h11 * h22 - h12 * h12;
  if (!(det > 0.0)) return;
  const double s1 = -(h22 * r1 - h12 * r2) / det, s2 = -(h11 * r2 - h12 * r1) / det;
  const int pix = Flist[k];
  const double d1 = fmin(fmax((double)delta[2 * pix] + s1, -(double)half_l), (double)half_l);
  const double d2 = fmin(fmax((double)delta[2 * pix + 1] + s2, -(double)half_m), (double)half_m);
  delta[2 * pix] = (float)d1;
  delta[2 * pix + 1] = (float)d2;
}

// bounds of the free pixels at their shifted directions: one wave per pixel,
// h = a^H M a with M = R^-1 (kind 0: gamma = C / h + kb / h) or M = R
// (kind 1: gamma = h (1 + kb)); kind 2: no bound
__global__ __launch_bounds__(256) void gamma_off_kernel(int kind, const float2* __restrict__ M, int P, int Pp,
                                                        const int* __restrict__ Flist, int n,
                                                        const float* __restrict__ xf, double C, double kb,
                                                        float* __restrict__ gamma) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (k >= n) return;
  const int pix = Flist[k];
  if (kind == 2) {
    if (lane == 0) gamma[pix] = INFINITY;
    return;
  }
  const float* a = xf + (size_t)k * 2 * Pp;
  double h = 0.0;
  for (int p = lane; p < P; p += 64) {
    float yr = 0.f, yi = 0.f;
    for (int q = 0; q < P; ++q) {
      const float2 e = M[p * P + q];
      const float ar = a[2 * q], ai = a[2 * q + 1];
      yr += e.x * ar - e.y * ai;
      yi += e.x * ai + e.y * ar;
    }
    h += (double)a[2 * p] * yr + (double)a[2 * p + 1] * yi;  // Re(conj(a_p) y_p)
  }
  h = wave_sum_dbl(h);
  if (lane != 0) return;
  gamma[pix] = (float)(kind == 0 ? C / h + kb / h : h * (1.0 + kb));
}

// offsets of pixels outside F back to zero; upper-set pixels at their on-grid bound
__global__ void offgrid_sets_kernel(const uint8_t* __restrict__ state, int Q, const float* __restrict__ gamma0,
                                    float* __restrict__ delta, float* __restrict__ sigma) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < Q; i += gridDim.x * blockDim.x) {
    const uint8_t s = state[i];
    if (s != 1) {
      delta[2 * i] = 0.f;
      delta[2 * i + 1] = 0.f;
    }
    if (s == 2) sigma[i] = gamma0[i];
  }
}

// ||M||_F^2 of a P x P complex matrix (one workgroup, FP64)
__global__ __launch_bounds__(256) void frob2_kernel(const float2* __restrict__ M, int n, double* out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) s += (double)M[e].x * M[e].x + (double)M[e].y * M[e].y;
  s = wave_sum_dbl(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

hipError_t launch_xf_off(const double* pos, int P, double lam, int nl, double l0, double dl, double m0, double dm,
                         const int* Flist, int n, const float* delta, float* xf, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int Pp = pad_p(P);
  const int grid = std::min((n * Pp + 255) / 256, 2048);
  hipLaunchKernelGGL(xf_off_kernel, dim3(grid), dim3(256), 0, st, pos, P, Pp, lam, nl, l0, dl, m0, dm, Flist, n,
                     delta, xf);
  return hipGetLastError();
}

hipError_t launch_newton_offset(const float2* E, int P, const double* pos, double lam, const int* Flist, int n,
                                const float* z, const float* xf, float* delta, float half_l, float half_m,
                                hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(newton_offset_kernel, dim3((n + 3) / 4), dim3(256), 0, st, E, P, pad_p(P), pos, lam, Flist, n,
                     z, xf, delta, half_l, half_m);
  return hipGetLastError();
}

hipError_t launch_gamma_off(int kind, const float2* M, int P, const int* Flist, int n, const float* xf, double C,
                            double kb, float* gamma, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gamma_off_kernel, dim3((n + 3) / 4), dim3(256), 0, st, kind, M, P, pad_p(P), Flist, n, xf, C,
                     kb, gamma);
  return hipGetLastError();
}

hipError_t launch_offgrid_sets(const uint8_t* state, int Q, const float* gamma0, float* delta, float* sigma,
                               hipStream_t st) {
  const int grid = std::min((Q + 255) / 256, 2048);
  hipLaunchKernelGGL(offgrid_sets_kernel, dim3(grid), dim3(256), 0, st, state, Q, gamma0, delta, sigma);
  return hipGetLastError();
}

hipError_t launch_frob2(const float2* M, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(frob2_kernel, dim3(1), dim3(256), 0, st, M, n, out);
  return hipGetLastError();
}

}  // namespace clsimg
