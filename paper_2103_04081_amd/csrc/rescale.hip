// Rescaling of the factor columns between steps.  The error analysis of the
// fixed-step method (Section 4.2) assumes bounded factors and remarks that
// scaling the factors after each iteration keeps them so, without a formula.
// The scaling used here leaves the CP model unchanged: rank component r has
// column norms nu_k = ||A^(k)(:, r)||, and each column is multiplied by
// g / nu_k with g = (prod_k nu_k)^(1/N), so all N columns end with norm g and
// the product of the scales is one.  A component with a zero or non-finite
// norm is left as it is.  One block per component; norms and scales in FP64
// with a fixed summation order, factors in FP32.
#include "cpd_runtime.hpp"

namespace cpdmi {

constexpr int kRescaleThreads = 256;
constexpr int kRescaleHeld = 2;  // column entries per thread kept in registers

__global__ void __launch_bounds__(kRescaleThreads) rescale_kernel(const ChainDesc* __restrict__ dp) {
  __shared__ double red[kMaxModes][kRescaleThreads];
  __shared__ double scale[kMaxModes];
  __shared__ int go;
  const int tid = threadIdx.x, r = blockIdx.x;
  const int N = dp->N, R = dp->R;
  // the sticky status is read together with the columns; nothing is
  // written unless it is clear
  if (tid == 0) go = dp->state->status == 0;
  // squared column norms of all modes at once: every mode's loads are in
  // flight together (the first kRescaleHeld entries of each thread stay in
  // registers for the scale pass), then one tree over the N partial sums
  float held[kMaxModes][kRescaleHeld];
#pragma unroll
  for (int k = 0; k < kMaxModes; ++k) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kRescaleHeld; ++j) held[k][j] = 0.f;
    if (k < N) {
      const CPD_GLOBAL float* Ak = gmem((const float*)dp->A[k]);
      const int I = dp->dims[k];
#pragma unroll
      for (int j = 0; j < kRescaleHeld; ++j) {
        const int i = tid + j * kRescaleThreads;
        if (i < I) held[k][j] = Ak[(int64_t)i * R + r];
      }
#pragma unroll
      for (int j = 0; j < kRescaleHeld; ++j) {
        const double v = held[k][j];
        s += v * v;
      }
      for (int i = tid + kRescaleHeld * kRescaleThreads; i < I; i += kRescaleThreads) {
        const double v = Ak[(int64_t)i * R + r];
        s += v * v;
      }
    }
    red[k][tid] = s;
  }
  __syncthreads();
  for (int h = kRescaleThreads / 2; h > 0; h >>= 1) {
    if (tid < h)
      for (int k = 0; k < N; ++k) red[k][tid] += red[k][tid + h];
    __syncthreads();
  }
  if (tid == 0) {
    bool ok = go != 0;
    double prod = 1.0;
    for (int k = 0; k < N; ++k) {
      scale[k] = sqrt(red[k][0]);
      ok = ok && isfinite(scale[k]) && scale[k] > 0.0;
      prod *= scale[k];
    }
    const double g = ok ? pow(prod, 1.0 / N) : 0.0;
    ok = ok && isfinite(g) && g > 0.0;
    for (int k = 0; k < N; ++k) scale[k] = ok ? g / scale[k] : 1.0;
    go = ok;
  }
  __syncthreads();
  if (!go) return;
#pragma unroll
  for (int k = 0; k < kMaxModes; ++k) {
    if (k < N) {
      CPD_GLOBAL float* Ak = gmem(dp->A[k]);
      const int I = dp->dims[k];
      const float sk = (float)scale[k];
#pragma unroll
      for (int j = 0; j < kRescaleHeld; ++j) {
        const int i = tid + j * kRescaleThreads;
        if (i < I) Ak[(int64_t)i * R + r] = held[k][j] * sk;
      }
      for (int i = tid + kRescaleHeld * kRescaleThreads; i < I; i += kRescaleThreads)
        Ak[(int64_t)i * R + r] *= sk;
    }
  }
}

hipError_t launch_rescale(const ChainDesc* d_desc, int R, hipStream_t stream) {
  hipLaunchKernelGGL(rescale_kernel, dim3(R), dim3(kRescaleThreads), 0, stream, d_desc);
  return hipGetLastError();
}

}  // namespace cpdmi
