// Prototype-filter design on the GPU (plan time).
//
// The PPF's coefficients come from a constant response function: the ideal
// rectangular pass band of one channel is a sinc in time, sampled, cut to
// T*N points and tapered by a window (section 2, the paragraphs after
// Eq. 1; the paper uses the Kaiser window). The value of coefficient j of
// a prototype of L = T*N points is
//
//     v[j] = w[j] * sinc((j - (L-1)/2) / N),   sinc(u) = sin(pi u)/(pi u),
//
// and the coefficients are v / sum(v), so that the gain at DC is 1.
// Everything is computed in FP64 and rounded once to FP32.

#include <hip/hip_runtime.h>

#include "../../include/ppf.h"
#include "ppf_internal.h"

namespace ppf {
namespace {

constexpr int kDesignBlock = 256;
constexpr int kSumBlock = 1024;

// Modified Bessel function of the first kind, order 0, from its power
// series sum_k ((x/2)^k / k!)^2; all terms are positive, so the sum is
// accurate to a few FP64 ulps. |x| <= 60 needs under 200 terms.
__device__ double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k <= 1000; ++k) {
    term = term * q / ((double)k * (double)k);
    sum += term;
    if (term <= sum * 1e-17) break;
  }
  return sum;
}

__global__ void __launch_bounds__(kDesignBlock)
ppf_design_values_kernel(double* v, int L, int N, int window, double beta, const double* user) {
  const long long j = (long long)blockIdx.x * kDesignBlock + threadIdx.x;
  if (j >= L) return;
  // 2j - (L-1) is an exact integer: twice the distance from the centre
  const double twice_off = 2.0 * (double)j - (double)(L - 1);
  double w = 1.0;
  if (window == PPF_WIN_USER) {
    w = user[j];
  } else if (L > 1) {
    const double a = (double)j / (double)(L - 1);              // j/(L-1)
    switch (window) {
      case PPF_WIN_HAMMING: w = 0.54 - 0.46 * cospi(2.0 * a); break;
      case PPF_WIN_HANN: w = 0.5 - 0.5 * cospi(2.0 * a); break;
      case PPF_WIN_KAISER: {
        const double r = twice_off / (double)(L - 1);           // 2j/(L-1) - 1
        const double s = 1.0 - r * r;
        w = bessel_i0(beta * sqrt(s > 0.0 ? s : 0.0)) / bessel_i0(beta);
        break;
      }
      default: w = 1.0; break;                                   // rectangular
    }
  }
  const double u = twice_off / (2.0 * (double)N);
  const double sinc = (twice_off == 0.0) ? 1.0 : sinpi(u) / (M_PI * u);
  v[j] = w * sinc;
}

// One block: the FP64 sum in a fixed order (thread i takes j = i, i+1024,
// ..., then a tree over the threads), then h = v / sum rounded to FP32.
__global__ void __launch_bounds__(kSumBlock)
ppf_design_normalise_kernel(const double* v, int L, float* h, double* sum_out) {
  __shared__ double part[kSumBlock];
  double s = 0.0;
  for (int j = threadIdx.x; j < L; j += kSumBlock) s += v[j];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = kSumBlock / 2; w > 0; w /= 2) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  const double total = part[0];
  for (int j = threadIdx.x; j < L; j += kSumBlock) h[j] = (float)(v[j] / total);
  if (threadIdx.x == 0) *sum_out = total;
}

}  // namespace

// v and h are device buffers of L doubles and L floats, sum one double;
// user is a device buffer of L doubles for PPF_WIN_USER, else unused.
hipError_t launch_design(int L, int N, int window, double beta, const double* user, double* v, float* h,
                         double* sum, hipStream_t st) {
  if (L <= 0 || N <= 0) return hipErrorInvalidValue;
  const int grid = (L + kDesignBlock - 1) / kDesignBlock;
  hipLaunchKernelGGL(ppf_design_values_kernel, dim3(grid), dim3(kDesignBlock), 0, st, v, L, N, window, beta, user);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ppf_design_normalise_kernel, dim3(1), dim3(kSumBlock), 0, st, (const double*)v, L, h, sum);
  return hipGetLastError();
}

}  // namespace ppf
