// Tensor layout (N mode-major copies) and the fit check.
//
// Layout: copy n holds X_(n)^T row-major, i.e. row j is the mode-n fibre at
// unfolding column j of the paper's index map (Section 1), padded to ld[n]
// elements so every fibre starts on a 128-byte boundary and is read in full
// cache lines by the step kernel.  Copy 0 is the dense tensor itself with
// padded rows; the other copies are batched transposes through LDS tiles.
//
// Fit (Section 5.2): Tol = ||[[A]] - X||^2 / ||X||^2 expanded as
//   (||X||^2 - 2 <X, [[A]]> + ||[[A]]||^2) / ||X||^2,
// with ||[[A]]||^2 = 1^T (hadamard_k A^(k)T A^(k)) 1 in FP64 and
// <X, [[A]]> = sum_j sum_i x_j(i) (A^(1)(i,:) . z_j) streamed over copy 0
// (z_j the KRP row of the fibre's multi-index), FP64 accumulation.
#include "cpd_internal.hpp"

namespace cpdmi {

template <typename T>
__device__ inline float load_as_f32(const T* p, int64_t i);
template <>
__device__ inline float load_as_f32<float>(const float* p, int64_t i) { return p[i]; }
template <>
__device__ inline float load_as_f32<double>(const double* p, int64_t i) { return (float)p[i]; }
template <>
__device__ inline float load_as_f32<uint16_t>(const uint16_t* p, int64_t i) {
  return bf16_to_f32(p[i]);
}

template <typename T>
__device__ inline void store_from_f32(T* p, int64_t i, float v);
template <>
__device__ inline void store_from_f32<float>(float* p, int64_t i, float v) { p[i] = v; }
template <>
__device__ inline void store_from_f32<uint16_t>(uint16_t* p, int64_t i, float v) {
  p[i] = f32_to_bf16_rne(v);
}

// Source element with dense linear index `lin` (mode 0 fastest): the source is
// either the dense tensor (sld = I0) or copy 0 (sld = ld[0]).
__device__ inline int64_t src_offset(int64_t lin, int I0, int64_t sld) {
  const int64_t rest = lin / I0;
  return (lin - rest * I0) + rest * sld;
}

// Copy 0 from a dense source: row j = elements [j*I0, (j+1)*I0).
template <typename Tin, typename Tout>
__global__ void layout_copy0(const Tin* __restrict__ src, Tout* __restrict__ dst, int I0,
                             int64_t rows, int ld) {
  const int64_t total = rows * I0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / I0;
    const int64_t i = e - j * I0;
    store_from_f32(dst, j * ld + i, load_as_f32(src, e));
  }
}

// Copy n >= 1: view the source as [b][i][a] (a < L = prod_{m<n} I_m fastest,
// i < In, b < U = prod_{m>n} I_m) and write dst[(a + L b) * ld + i].
template <typename Tin, typename Tout>
__global__ void layout_transpose(const Tin* __restrict__ src, Tout* __restrict__ dst, int I0,
                                 int64_t sld, int64_t L, int In, int64_t U, int ld) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t ntA = (L + 31) / 32, ntI = (In + 31) / 32;
  const int64_t ntiles = ntA * ntI * U;
  for (int64_t tidx = blockIdx.x; tidx < ntiles; tidx += gridDim.x) {
    const int64_t b = tidx / (ntA * ntI);
    const int64_t r = tidx - b * ntA * ntI;
    const int64_t ta = r % ntA, ti = r / ntA;
    const int64_t a0 = ta * 32, i0 = ti * 32;
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
      const int64_t a = a0 + tx, i = i0 + k;
      float v = 0.f;
      if (a < L && i < In) v = load_as_f32(src, src_offset(a + L * (i + (int64_t)In * b), I0, sld));
      tile[k][tx] = v;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
      const int64_t a = a0 + k, i = i0 + tx;
      if (a < L && i < In) store_from_f32(dst, (a + L * b) * ld + i, tile[tx][k]);
    }
  }
}

template <typename Tin, typename Tout>
static hipError_t layout_all(const Tin* src, bool src_is_copy0, const ChainDesc& d, int nmodes_from,
                             hipStream_t stream) {
  const int N = d.N;
  const int I0 = d.dims[0];
  int64_t total = 1;
  for (int k = 0; k < N; ++k) total *= d.dims[k];
  const int64_t sld = src_is_copy0 ? d.ld[0] : I0;
  if (nmodes_from == 0) {
    const int64_t rows = total / I0;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((layout_copy0<Tin, Tout>), dim3((unsigned)blocks), dim3(256), 0, stream, src,
                       (Tout*)d.X[0], I0, rows, d.ld[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  int64_t L = I0;
  for (int n = 1; n < N; ++n) {
    const int In = d.dims[n];
    const int64_t U = total / (L * In);
    const int64_t tiles = ((L + 31) / 32) * ((In + 31) / 32) * U;
    const unsigned blocks = (unsigned)(tiles < 65536 ? tiles : 65536);
    hipLaunchKernelGGL((layout_transpose<Tin, Tout>), dim3(blocks), dim3(256), 0, stream, src,
                       (Tout*)d.X[n], I0, sld, L, In, U, d.ld[n]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    L *= In;
  }
  return hipSuccess;
}

// Build every copy from a dense device tensor of type in_dtype (F32 or F64).
hipError_t launch_layout_from_dense(const void* X, int in_dtype, const ChainDesc& d,
                                    hipStream_t stream) {
  if (d.dtype == CPD_BF16) {
    if (in_dtype == CPD_F64) return layout_all<double, uint16_t>((const double*)X, false, d, 0, stream);
    return layout_all<float, uint16_t>((const float*)X, false, d, 0, stream);
  }
  if (in_dtype == CPD_F64) return layout_all<double, float>((const double*)X, false, d, 0, stream);
  return layout_all<float, float>((const float*)X, false, d, 0, stream);
}

// Build copies 1..N-1 from copy 0 (already in storage type).
hipError_t launch_layout_from_copy0(const ChainDesc& d, hipStream_t stream) {
  if (d.dtype == CPD_BF16)
    return layout_all<uint16_t, uint16_t>((const uint16_t*)d.X[0], true, d, 1, stream);
  return layout_all<float, float>((const float*)d.X[0], true, d, 1, stream);
}

// ---------------------------------------------------------------------------
// Fit: partial sums over the rows of copy 0.  mode 0: sum x^2; mode 1:
// sum_j sum_i x_j(i) * (A^(0)(i,:) . z_j).  One partial per block.
// ---------------------------------------------------------------------------
template <typename T, bool INNER>
__global__ void __launch_bounds__(kFitBlock) fit_partial_kernel(const ChainDesc* __restrict__ descs,
                                                                int nparts_per_chain, int a0_in_lds) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[kFitBlock / 64];
  const ChainDesc* dp = descs + blockIdx.y;
  if (!dp->active || (INNER && dp->state->done)) return;
  const int N = dp->N, R = dp->R, I0 = dp->dims[0], ld0 = dp->ld[0];
  const T* X0 = (const T*)dp->X[0];
  // A^(1) rows: staged in LDS when they fit, else read through the caches
  const float* A0s = a0_in_lds ? (const float*)smem : dp->A[0];
  if (INNER && a0_in_lds) {
    float* dst = (float*)smem;
    for (int e = threadIdx.x; e < I0 * R; e += blockDim.x) dst[e] = dp->A[0][e];
    __syncthreads();
  }
  int64_t rows = 1;
  for (int k = 1; k < N; ++k) rows *= dp->dims[k];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wpb = kFitBlock / 64;
  const int64_t gw = (int64_t)blockIdx.x * wpb + wave, nw = (int64_t)nparts_per_chain * wpb;
  double acc = 0.0;
  for (int64_t j = gw; j < rows; j += nw) {
    const T* xr = X0 + j * ld0;
    if (!INNER) {
      for (int i = lane; i < I0; i += 64) {
        const double x = (double)load_as_f32(xr, i);
        acc += x * x;
      }
    } else {
      // z_j(r) for r = lane (lanes >= R idle); R <= 64
      float z = 0.f;
      if (lane < R) {
        int64_t rem = j;
        z = 1.f;
        for (int k = 1; k < N; ++k) {
          const int ik = (int)(rem % dp->dims[k]);
          rem /= dp->dims[k];
          z *= dp->A[k][(int64_t)ik * R + lane];
        }
      }
      for (int i0 = 0; i0 < I0; i0 += 64) {
        const int i = i0 + lane;
        float v = 0.f;
        for (int r = 0; r < R; ++r) {
          const float zr = __shfl(z, r);
          if (i < I0) v = fmaf(A0s[i * R + r], zr, v);
        }
        if (i < I0) acc += (double)load_as_f32(xr, i) * (double)v;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < wpb; ++w) s += red[w];
    dp->parts[blockIdx.x] = s;
  }
}

// Final reduction (one block per chain).  mode 0: state->x2 = sum of parts.
// mode 1: inner product, ||[[A]]||^2 from the Grams, and the fit.
template <bool INNER>
__global__ void __launch_bounds__(1024) fit_final_kernel(const ChainDesc* __restrict__ descs,
                                                         int nparts_per_chain) {
  __shared__ double red[16];
  const ChainDesc* dp = descs + blockIdx.x;
  if (!dp->active || (INNER && dp->state->done)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double s = 0.0;
  for (int p = threadIdx.x; p < nparts_per_chain; p += blockDim.x) s += dp->parts[p];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  double total = 0.0;
  for (int w = 0; w < (int)(blockDim.x / 64); ++w) total += red[w];
  __syncthreads();
  if (!INNER) {
    if (threadIdx.x == 0) dp->state->x2 = total;
    return;
  }
  // ||[[A]]||^2 = sum_{r,s} prod_k (A^(k)T A^(k))_{rs}
  const int R = dp->R, N = dp->N;
  double h = 0.0;
  for (int pr = threadIdx.x; pr < R * R; pr += blockDim.x) {
    const int r = pr / R, c = pr - r * R;
    double prod = 1.0;
    for (int k = 0; k < N; ++k) {
      const float* A = dp->A[k];
      double g = 0.0;
      for (int i = 0; i < dp->dims[k]; ++i) g += (double)A[(int64_t)i * R + r] * (double)A[(int64_t)i * R + c];
      prod *= g;
    }
    h += prod;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o);
  if (lane == 0) red[wave] = h;
  __syncthreads();
  if (threadIdx.x == 0) {
    double xh = 0.0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) xh += red[w];
    ChainState* st = dp->state;
    st->inner = total;
    st->xhat2 = xh;
    st->fit = 1.0 - (st->x2 - 2.0 * total + xh) / st->x2;
    if (dp->autostop && ((dp->fit_target > 0.0 && st->fit >= dp->fit_target) ||
                         (dp->step_limit > 0 && st->t >= dp->step_limit) || st->status != 0)) {
      st->done = 1;
      st->t_done = st->t;
      st->clock_done = (int64_t)wall_clock64();
    }
  }
}

constexpr size_t kFitLdsMax = 64 * 1024;

hipError_t launch_fit(const ChainDesc* d_descs, int nchains, int dtype, int max_I0, int max_R,
                      bool inner, hipStream_t stream) {
  const size_t need = sizeof(float) * (size_t)max_I0 * max_R;
  const int in_lds = inner && need <= kFitLdsMax;
  const size_t lds = in_lds ? need : 0;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)fit_partial_kernel<float, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kFitLdsMax);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)fit_partial_kernel<uint16_t, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kFitLdsMax);
    if (e != hipSuccess) return e;
    attr = true;
  }
  dim3 grid(kFitParts, nchains);
  if (dtype == CPD_BF16) {
    if (inner)
      hipLaunchKernelGGL((fit_partial_kernel<uint16_t, true>), grid, dim3(kFitBlock), lds, stream,
                         d_descs, kFitParts, in_lds);
    else
      hipLaunchKernelGGL((fit_partial_kernel<uint16_t, false>), grid, dim3(kFitBlock), 0, stream,
                         d_descs, kFitParts, 0);
  } else {
    if (inner)
      hipLaunchKernelGGL((fit_partial_kernel<float, true>), grid, dim3(kFitBlock), lds, stream,
                         d_descs, kFitParts, in_lds);
    else
      hipLaunchKernelGGL((fit_partial_kernel<float, false>), grid, dim3(kFitBlock), 0, stream,
                         d_descs, kFitParts, 0);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (inner)
    hipLaunchKernelGGL((fit_final_kernel<true>), dim3(nchains), dim3(1024), 0, stream, d_descs,
                       kFitParts);
  else
    hipLaunchKernelGGL((fit_final_kernel<false>), dim3(nchains), dim3(1024), 0, stream, d_descs,
                       kFitParts);
  return hipGetLastError();
}

}  // namespace cpdmi
