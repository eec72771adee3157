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
#include <algorithm>

#include "cpd_runtime.hpp"

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

// Copy 0 from the dense tensor already in the storage type (staged on the
// device without row padding).
hipError_t launch_copy0_from_staged(const void* staged, const ChainDesc& d, hipStream_t stream) {
  int64_t total = 1;
  for (int k = 0; k < d.N; ++k) total *= d.dims[k];
  const int I0 = d.dims[0];
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (d.dtype == CPD_BF16)
    hipLaunchKernelGGL((layout_copy0<uint16_t, uint16_t>), dim3((unsigned)blocks), dim3(256), 0,
                       stream, (const uint16_t*)staged, (uint16_t*)d.X[0], I0, total / I0, d.ld[0]);
  else
    hipLaunchKernelGGL((layout_copy0<float, float>), dim3((unsigned)blocks), dim3(256), 0, stream,
                       (const float*)staged, (float*)d.X[0], I0, total / I0, d.ld[0]);
  return hipGetLastError();
}

// Build copies 1..N-1 from copy 0 (already in storage type).
hipError_t launch_layout_from_copy0(const ChainDesc& d, hipStream_t stream) {
  if (d.dtype == CPD_BF16)
    return layout_all<uint16_t, uint16_t>((const uint16_t*)d.X[0], true, d, 1, stream);
  return layout_all<float, float>((const float*)d.X[0], true, d, 1, stream);
}

// ---------------------------------------------------------------------------
// Fit, partial pass over copy 0 (row j = the mode-1 fibre j, I0 elements).
//   norm pass:  sum_j sum_i x_j(i)^2
//   inner pass: sum_j sum_r z_j(r) y_j(r),  y_j = x_j A^(1)  (1 x R),
//               z_j(r) = prod_{k>0} A^(k)(i_k(j), r)
// Each block owns a contiguous range of rows; its four waves take 16-row
// tiles in turn.  y for a tile is a 16 x I0 by I0 x R product on
// v_mfma_f32_16x16x4f32 (the tensor's BF16 or FP32 values as the A
// operand, A^(1) in FP32 as the B operand, FP32 accumulation), with A^(1)
// staged transposed in LDS when it fits.  Per-tile sums are accumulated in
// FP64.  Which block serves which decomposition comes from a prefix table
// (start[c] = first block of decomposition c), so one launch covers a batch.
// ---------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));
typedef uint32_t w4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ void unpack16(const w4& v, float* x);
template <>
__device__ __forceinline__ void unpack16<float>(const w4& v, float* x) {
  x[0] = __uint_as_float(v[0]);
  x[1] = __uint_as_float(v[1]);
  x[2] = __uint_as_float(v[2]);
  x[3] = __uint_as_float(v[3]);
}
template <>
__device__ __forceinline__ void unpack16<uint16_t>(const w4& v, float* x) {
  const uint32_t w[4] = {v[0], v[1], v[2], v[3]};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    x[2 * q] = __uint_as_float(w[q] << 16);
    x[2 * q + 1] = __uint_as_float(w[q] & 0xFFFF0000u);
  }
}

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Row stride (elements) of the BF16 copies of A^(1) the BF16 inner pass
// stages in LDS: a multiple of 64 columns plus 8 (16-byte aligned rows whose
// 16 rank columns start in distinct banks).
__host__ __device__ inline int fit_a0_stride16(int I0) { return (I0 + 63) / 64 * 64 + 8; }

__device__ __forceinline__ int fit_chain_of(const int32_t* start, int nchains, int bid) {
  int lo = 0, hi = nchains;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= bid) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Inner pass over the ranks [r_off, r_off + 64) (up to four rank tiles);
// R > 64 takes a second pass (r_off = 64) whose sums are added to the first's.
template <typename T, bool INNER>
__global__ void __launch_bounds__(kFitBlock) __attribute__((amdgpu_waves_per_eu(4))) fit_partial_kernel(const ChainDesc* __restrict__ descs,
                                                                const int32_t* __restrict__ start,
                                                                int nchains, int lds_floats,
                                                                int r_off) {
  extern __shared__ __align__(16) float a0t[];
  __shared__ double red[kFitBlock / 64];
  constexpr int E = 16 / (int)sizeof(T);  // elements per 16-byte load
  constexpr int U = 64 / (4 * E);         // loads per lane per 64 columns
  constexpr int Q = 4 * (int)sizeof(T);   // 16-byte words per 64 columns
  const int c = fit_chain_of(start, nchains, blockIdx.x);
  const ChainDesc* dp = descs + c;
  if (!dp->active || (INNER && dp->state->done)) return;
  const int b = blockIdx.x - start[c], nb = start[c + 1] - start[c];
  const int N = dp->N, R = dp->R, I0 = dp->dims[0], ld0 = dp->ld[0];
  int64_t J0 = 1;
  for (int k = 1; k < N; ++k) J0 *= dp->dims[k];
  const int64_t rpb = ((J0 + nb - 1) / nb + 15) / 16 * 16;
  const int64_t r0 = (int64_t)b * rpb;
  const int64_t r1 = r0 + rpb < J0 ? r0 + rpb : J0;
  if (INNER && r_off >= R) return;  // a second pass only for R > 64
  const int RT = min(4, (R - r_off + 15) / 16);
  const int P = fit_a0_stride(I0);
  // BF16 storage: the stored values feed v_mfma_f32_16x16x32_bf16 directly,
  // A^(1) = hi + lo as two BF16 terms (16 significant bits; products exact
  // in FP32), staged transposed in LDS
  constexpr bool kBf16 = sizeof(T) == 2;
  const int P16 = fit_a0_stride16(I0);
  const bool in_lds16 = INNER && kBf16 && 2 * 16 * RT * P16 <= 2 * lds_floats;
  const bool in_lds = INNER && !in_lds16 && 16 * RT * P <= lds_floats;
  uint16_t* a0h = (uint16_t*)a0t;
  uint16_t* a0l = a0h + 16 * RT * P16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rq = lane & 15, kg = lane >> 4;
  const CPD_GLOBAL float* A0 = gmem((const float*)dp->A[0]);
  const CPD_GLOBAL char* X0 = gmem((const char*)dp->X[0]);
  w4 va[U], vb[U];  // inner pass: chunk buffers, the first one carried across tiles
  if (INNER && r0 + 16 * wave < r1) {
    // the wave's first chunk is in flight while A^(1) is staged
    const int64_t t0 = r0 + 16 * wave;
    const int64_t jr = t0 + rq < J0 ? t0 + rq : J0 - 1;
    const CPD_GLOBAL w4* xr = (const CPD_GLOBAL w4*)(X0 + jr * (int64_t)ld0 * sizeof(T));
#pragma unroll
    for (int u = 0; u < U; ++u) va[u] = xr[4 * u + kg];
  }
  if (in_lds) {
    for (int e = tid; e < 16 * RT * P; e += kFitBlock) a0t[e] = 0.f;
    __syncthreads();
    for (int e = tid; e < I0 * R; e += kFitBlock) {
      const int i = e / R, col = e - i * R - r_off;
      if (col >= 0 && col < 16 * RT) a0t[col * P + i] = A0[e];
    }
    __syncthreads();
  }
  if (in_lds16) {
    for (int e = tid; e < 2 * 16 * RT * P16; e += kFitBlock) a0h[e] = 0;
    __syncthreads();
    for (int e = tid; e < I0 * R; e += kFitBlock) {
      const int i = e / R, col = e - i * R - r_off;
      if (col < 0 || col >= 16 * RT) continue;
      const float v = A0[e];
      const uint16_t h = f32_to_bf16_rne(v);
      a0h[col * P16 + i] = h;
      a0l[col * P16 + i] = f32_to_bf16_rne(v - bf16_to_f32(h));
    }
    __syncthreads();
  }
  const bool small_rows = J0 < ((int64_t)1 << 31);
  const int nit = (I0 + 63) / 64;
  double accd = 0.0;
  for (int64_t t0 = r0 + 16 * wave; t0 < r1; t0 += 16 * (kFitBlock / 64)) {
    const int64_t jr = t0 + rq < J0 ? t0 + rq : J0 - 1;  // rows past the end: any valid row
    const CPD_GLOBAL w4* xr = (const CPD_GLOBAL w4*)(X0 + jr * (int64_t)ld0 * sizeof(T));
    if (!INNER) {
      const bool row_ok = t0 + rq < r1;
      for (int it = 0; it < nit; ++it) {
        w4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = xr[it * Q + 4 * u + kg];
        float sq = 0.f;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          float x[E];
          unpack16<T>(v[u], x);
#pragma unroll
          for (int s2 = 0; s2 < E; ++s2) sq = fmaf(x[s2], x[s2], sq);
        }
        if (row_ok) accd += (double)sq;
      }
      continue;
    }
    f4 acc[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) acc[rt] = f4{0.f, 0.f, 0.f, 0.f};
    auto compute = [&](const w4 (&v)[U], int it) {
      if constexpr (kBf16) {
        if (in_lds16) {
          // K block of 32 columns per 16-byte load: lane group kg holds
          // columns 8 kg .. 8 kg + 7 of it, the A operand as stored
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const bf8 a = __builtin_bit_cast(bf8, v[u]);
            const int ib = 64 * it + 32 * u + 8 * kg;
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
              if (rt < RT) {
                const int o = (16 * rt + rq) * P16 + ib;
                const bf8 bh = __builtin_bit_cast(bf8, *(const w4*)(a0h + o));
                const bf8 bl = __builtin_bit_cast(bf8, *(const w4*)(a0l + o));
                acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, acc[rt], 0, 0, 0);
                acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc[rt], 0, 0, 0);
              }
            }
          }
          return;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        float x[E];
        unpack16<T>(v[u], x);
        const int ib = 64 * it + (4 * u + kg) * E;  // column of x[0]
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
          if (rt < RT) {
            const int col = 16 * rt + rq;   // relative to r_off
#pragma unroll
            for (int s4 = 0; s4 < E / 4; ++s4) {
              f4 bv;
              if (in_lds) {
                bv = *(const f4*)(a0t + col * P + ib + 4 * s4);
              } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                  const int i = ib + 4 * s4 + s;
                  bv[s] = (i < I0 && r_off + col < R) ? A0[(int64_t)i * R + r_off + col] : 0.f;
                }
              }
#pragma unroll
              for (int s = 0; s < 4; ++s)
                acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[4 * s4 + s], bv[s], acc[rt], 0, 0, 0);
            }
          }
        }
      }
    };
    // The epilogue's factor entries, loaded now so that their round trips
    // overlap the products.  Lane (kg, rq) holds y of rows jb..jb+3 (jb =
    // t0 + 4 kg), column 16 rt + rq.  z_j = A^(2)(i_2) (x) w with w the
    // product over the higher modes, shared by the four rows unless i_2
    // wraps inside them (then the row takes the general path at the end);
    // A^(2) rows and the entries of modes 3 and 4 are prefetched, higher
    // modes (five-way and beyond) are loaded in the epilogue.
    const int64_t jb = t0 + 4 * kg;
    const int I1 = dp->dims[1];
    int i1b;
    int64_t hi;
    if (small_rows) {
      const uint32_t h = (uint32_t)jb / (uint32_t)I1;
      i1b = (int)((uint32_t)jb - h * (uint32_t)I1);
      hi = h;
    } else {
      hi = jb / I1;
      i1b = (int)(jb - hi * I1);
    }
    int colc[4];  // the lane's rank columns, clamped into the row (zeros selected after)
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int col = r_off + 16 * rt + rq;
      colc[rt] = col < R ? col : R - 1;
    }
    float wpre[2][4];
    int64_t hrem = hi;
#pragma unroll
    for (int k2 = 0; k2 < 2; ++k2) {
      const int k = 2 + k2;
      if (k < N) {
        const int Ik = dp->dims[k];
        const int64_t nxt = small_rows ? (int64_t)((uint32_t)hrem / (uint32_t)Ik) : hrem / Ik;
        const int ik = (int)(hrem - nxt * Ik);
        hrem = nxt;
        const CPD_GLOBAL float* Ak = gmem((const float*)dp->A[k]) + (int64_t)ik * R;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) wpre[k2][rt] = Ak[colc[rt]];
      }
    }
    float a1pre[4][4];
    {
      const CPD_GLOBAL float* A1 = gmem((const float*)dp->A[1]);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i1 = i1b + q < I1 ? i1b + q : I1 - 1;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) a1pre[q][rt] = A1[(int64_t)i1 * R + colc[rt]];
      }
    }
    // the first chunk of this wave's next tile is loaded during the last
    // chunk and the epilogue of this one
    const int64_t tn = t0 + 16 * (kFitBlock / 64);
    const CPD_GLOBAL w4* xn = (const CPD_GLOBAL w4*)(X0 + (tn + rq < J0 ? tn + rq : J0 - 1) *
                                                          (int64_t)ld0 * sizeof(T));
    for (int it = 0; it < nit; it += 2) {
      if (it + 1 < nit) {
#pragma unroll
        for (int u = 0; u < U; ++u) vb[u] = xr[(it + 1) * Q + 4 * u + kg];
      }
      compute(va, it);
      if (it + 2 < nit) {
#pragma unroll
        for (int u = 0; u < U; ++u) va[u] = xr[(it + 2) * Q + 4 * u + kg];
      } else if (tn < r1) {
#pragma unroll
        for (int u = 0; u < U; ++u) va[u] = xn[4 * u + kg];
      }
      if (it + 1 < nit) compute(vb, it + 1);
    }
    float part = 0.f;
    float w[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int col = r_off + 16 * rt + rq;
      float v = 1.f;
      if (N > 2) v *= wpre[0][rt];
      if (N > 3) v *= wpre[1][rt];
      w[rt] = (rt < RT && col < R) ? v : 0.f;
    }
    {
      int64_t rem = hrem;
      for (int k = 4; k < N; ++k) {
        const int Ik = dp->dims[k];
        const int64_t nxt = small_rows ? (int64_t)((uint32_t)rem / (uint32_t)Ik) : rem / Ik;
        const int ik = (int)(rem - nxt * Ik);
        rem = nxt;
        const CPD_GLOBAL float* Ak = gmem((const float*)dp->A[k]) + (int64_t)ik * R;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) w[rt] *= Ak[colc[rt]];
      }
    }
    const CPD_GLOBAL float* A1 = gmem((const float*)dp->A[1]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t j = jb + q;
      if (j < r1) {
        float z[4];
        const int i1 = i1b + q;
        if (i1 < I1) {
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) z[rt] = a1pre[q][rt] * w[rt];
        } else {
          // i_2 wrapped: the general multi-index of row j
          int64_t rem = j;
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) z[rt] = 1.f;
          for (int k = 1; k < N; ++k) {
            const int Ik = dp->dims[k];
            const int64_t nxt = rem / Ik;
            const int ik = (int)(rem - nxt * Ik);
            rem = nxt;
            const CPD_GLOBAL float* Ak = gmem((const float*)dp->A[k]) + (int64_t)ik * R;
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
              const int col = r_off + 16 * rt + rq;
              if (rt < RT) z[rt] *= col < R ? Ak[col] : 0.f;
            }
          }
        }
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
          if (rt < RT) part = fmaf(z[rt], acc[rt][q], part);
      }
    }
    accd += (double)part;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) accd += __shfl_xor(accd, o);
  if (lane == 0) red[wave] = accd;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int w = 0; w < kFitBlock / 64; ++w) sum += red[w];
    dp->parts[b] = r_off ? dp->parts[b] + sum : sum;
  }
}

// The fit from <X, [[A]]> (total) and the 16 wave sums of ||[[A]]||^2 in
// red (thread 0 of the final kernel), and the automatic stop.
__device__ inline void finish_fit(const ChainDesc* dp, double total, const double* red) {
  double xh = 0.0;
  for (int w = 0; w < 16; ++w) xh += red[w];
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

// Final reduction, one block per decomposition.  Norm pass: state->x2.
// Inner pass: <X, [[A]]>, ||[[A]]||^2 from the Gram matrices (FP64, rows
// split over threads, combined in a fixed order) and the fit.
template <bool INNER>
__global__ void __launch_bounds__(1024) fit_final_kernel(const ChainDesc* __restrict__ descs,
                                                         const int32_t* __restrict__ start) {
  __shared__ double red[16];
  __shared__ double had[4096];  // Hadamard products (R <= 64)
  __shared__ double slice[1024];
  const ChainDesc* dp = descs + blockIdx.x;
  if (!dp->active || (INNER && dp->state->done)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = start[blockIdx.x + 1] - start[blockIdx.x];
  // the partial sums p = tid, tid + 1024, ... (loaded now, summed when
  // needed: the small-R inner pass forms the Grams meanwhile)
  static_assert(kFitParts <= 4 * 1024, "four partials per thread");
  double pv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int p = tid + 1024 * q;
    const double v = dp->parts[p < nb ? p : 0];
    pv[q] = p < nb ? v : 0.0;
  }
  auto sum_parts = [&]() {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) s += pv[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) t += red[w];
    __syncthreads();
    return t;
  };
  if (!INNER) {
    const double total = sum_parts();
    if (tid == 0) dp->state->x2 = total;
    return;
  }
  const int R = dp->R, N = dp->N, R2 = R * R;
  __shared__ float rows[64 * kMaxRank];
  if (R <= 64) {
    // Up to four rank tiles: the modes' Grams on the FP64 matrix cores
    // (v_mfma_f64_16x16x4f64), tile (rt, ct) of G_k = A^(k)T A^(k) with lane
    // l holding A^(k)(4s + l/16, 16 rt + l % 16) as the A operand and
    // A^(k)(4s + l/16, 16 ct + l % 16) as the B operand for K-step s; element
    // q of lane l's result is G_k(16 rt + 4q + l/16, 16 ct + l % 16).  The
    // items (mode k, tile t, K-part p), p fastest, kp a power of two with
    // N T kp <= 16 where it can be, go to the 16 waves in rounds of 16 (one
    // round for small R: every mode's loads in flight together, straight
    // from global memory).  Per round the items' tiles go to LDS and each
    // element of had (the Hadamard product over the modes) is multiplied by
    // its (k, t) groups' part sums, in item order.  Ranks past R load zeros,
    // so their Gram entries and products are zero.
    typedef double d4 __attribute__((ext_vector_type(4)));
    double* part = (double*)rows;  // 16 x 256 doubles
    const int RT = (R + 15) / 16, T = RT * RT;
    int kp = 1;
    while (2 * kp * N * T <= 16) kp *= 2;
    const int nitems = N * T * kp;
    const int rq = lane & 15, kq = lane >> 4;
    for (int e = tid; e < T * 256; e += blockDim.x) had[e] = 1.0;
    const int wv = __builtin_amdgcn_readfirstlane(wave);  // uniform: the items' loops are scalar
    for (int r0 = 0; r0 < nitems; r0 += 16) {
      const int item = r0 + wv;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      if (item < nitems) {
        const int kpart = item % kp, kt = item / kp;
        const int k = kt / T, tile = kt - k * T;
        const int rt = tile / RT, ct = tile - rt * RT;
        const int ra = 16 * rt + rq, rb = 16 * ct + rq;
        // loads clamped into the factor and issued unconditionally (several
        // in flight); out-of-range entries are replaced by zeros after
        const int rac = ra < R ? ra : R - 1, rbc = rb < R ? rb : R - 1;
        const CPD_GLOBAL float* A = gmem((const float*)dp->A[k]);
        const int Ik = dp->dims[k], nks = (Ik + 3) >> 2;
        auto kstep = [&](int st, float& va, float& vb) {
          const int i = 4 * st + kq;
          const int64_t row = (int64_t)(i < Ik ? i : Ik - 1) * R;
          va = A[row + rac];
          vb = A[row + rbc];
        };
        auto mac = [&](int st, float va, float vb) {
          const int i = 4 * st + kq;
          const double xa = (i < Ik && ra < R) ? (double)va : 0.0;
          const double xb = (i < Ik && rb < R) ? (double)vb : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, xb, acc, 0, 0, 0);
        };
        // eight K-steps' loads in flight before their products
        int st = kpart;
        for (; st + 7 * kp < nks; st += 8 * kp) {
          float va[8], vb[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) kstep(st + u * kp, va[u], vb[u]);
#pragma unroll
          for (int u = 0; u < 8; ++u) mac(st + u * kp, va[u], vb[u]);
        }
        for (; st < nks; st += kp) {
          float va, vb;
          kstep(st, va, vb);
          mac(st, va, vb);
        }
      }
      __syncthreads();  // the previous round's tiles are consumed
      if (item < nitems) {
#pragma unroll
        for (int q = 0; q < 4; ++q) part[wv * 256 + (4 * q + kq) * 16 + rq] = acc[q];
      }
      __syncthreads();
      for (int e = tid; e < T * 256; e += blockDim.x) {
        const int te = e >> 8, o = e & 255;
        for (int g0 = r0; g0 < r0 + 16 && g0 < nitems; g0 += kp) {
          if ((g0 / kp) % T != te) continue;
          double gk = 0.0;
          for (int p2 = 0; p2 < kp; ++p2) gk += part[(g0 - r0 + p2) * 256 + o];
          had[e] *= gk;
        }
      }
    }
    __syncthreads();
    const double total = sum_parts();
    double h = 0.0;
    for (int e = tid; e < T * 256; e += blockDim.x) h += had[e];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o);
    if (lane == 0) red[wave] = h;
    __syncthreads();
    if (tid == 0) finish_fit(dp, total, red);
    return;
  }
  const double total = sum_parts();
  // ||[[A]]||^2 = sum_{r,c} prod_k (A^(k)T A^(k))_{rc}.  The factors pass
  // through LDS in chunks of as many rows as the buffer holds (a whole
  // factor at small R), mode after mode; the next chunk is loaded into
  // registers while the current one is summed, so the chunks' round trips
  // to memory overlap the sums.  Thread (pair p, slice sl) sums rows sl,
  // sl + slices, ... of the chunk for its pair in FP64 (two accumulators,
  // even and odd steps); slices combine in order.  With R^2 >= 1024 pairs
  // every thread owns the pairs tid + 1024 q (one accumulator each) and
  // keeps their Hadamard products in registers.
  const int slices = R2 >= 1024 ? 1 : 1024 / R2;
  constexpr int kRowBuf = 64 * kMaxRank;  // floats
  constexpr int kPer = kRowBuf / 1024;    // floats of the next chunk per thread
  constexpr int kPq = (kMaxRank * kMaxRank + 1023) / 1024;  // pairs per thread
  const int chunk = kRowBuf / R;  // rows per chunk
  double hp[kPq];
#pragma unroll
  for (int q = 0; q < kPq; ++q) hp[q] = 1.0;
  for (int p = tid; p < R2 && slices > 1; p += blockDim.x) had[p] = 1.0;
  float nx[kPer];
  auto fetch = [&](int k, int i0) {
    const CPD_GLOBAL float* A = gmem((const float*)dp->A[k]) + (int64_t)i0 * R;
    const int n = (dp->dims[k] - i0 < chunk ? dp->dims[k] - i0 : chunk) * R;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + 1024 * q;
      nx[q] = e < n ? A[e] : 0.f;
    }
  };
  double g[kPq];  // pairs tid + 1024 q (slices == 1)
#pragma unroll
  for (int q = 0; q < kPq; ++q) g[q] = 0.0;
  double gs = 0.0;  // pair tid % R2, slice tid / R2
  fetch(0, 0);
  for (int k = 0, i0 = 0; k < N;) {
    const int Ik = dp->dims[k];
    const int nr = Ik - i0 < chunk ? Ik - i0 : chunk;
    __syncthreads();  // the previous chunk is summed
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + 1024 * q;
      if (e < nr * R) rows[e] = nx[q];
    }
    __syncthreads();
    int kn = k, in = i0 + chunk;
    if (in >= Ik) {
      kn = k + 1;
      in = 0;
    }
    if (kn < N) fetch(kn, in);
    if (slices == 1) {
#pragma unroll
      for (int q = 0; q < kPq; ++q) {
        const int p = tid + q * 1024;
        if (p < R2) {
          // up to 16 pairs per thread: independent sums enough
          const int r = p / R, cc = p - r * R;
#pragma unroll 1
          for (int i = 0; i < nr; ++i) g[q] += (double)rows[i * R + r] * (double)rows[i * R + cc];
        }
      }
    } else {
      const int p = tid % R2, sl = tid / R2;
      if (sl < slices) {
        const int r = p / R, cc = p - r * R;
        double a0 = 0.0, a1 = 0.0;
        int i = sl;
        for (; i + slices < nr; i += 2 * slices) {
          a0 += (double)rows[i * R + r] * (double)rows[i * R + cc];
          a1 += (double)rows[(i + slices) * R + r] * (double)rows[(i + slices) * R + cc];
        }
        if (i < nr) a0 += (double)rows[i * R + r] * (double)rows[i * R + cc];
        gs += a0 + a1;
      }
    }
    if (kn != k) {
      // mode k complete: its Gram into the Hadamard products
      if (slices == 1) {
#pragma unroll
        for (int q = 0; q < kPq; ++q) {
          if (tid + q * 1024 < R2) hp[q] *= g[q];
          g[q] = 0.0;
        }
      } else {
        if (tid / R2 < slices) slice[tid] = gs;
        gs = 0.0;
        __syncthreads();
        if (tid < R2) {
          double t = 0.0;
          for (int q = 0; q < slices; ++q) t += slice[q * R2 + tid];
          had[tid] *= t;
        }
      }
    }
    k = kn;
    i0 = in;
  }
  __syncthreads();
  double h = 0.0;
  if (slices == 1) {
#pragma unroll
    for (int q = 0; q < kPq; ++q)
      if (tid + q * 1024 < R2) h += hp[q];
  } else {
    for (int p = tid; p < R2; p += blockDim.x) h += had[p];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o);
  if (lane == 0) red[wave] = h;
  __syncthreads();
  if (tid == 0) finish_fit(dp, total, red);
}

constexpr size_t kFitLightLds = 32 * 1024;  // groups the inner pass by staged LDS

FitPlan plan_fit(const ChainDesc* descs, int nchains, int32_t* tables) {
  FitPlan fp{{0, 0}, {0, 0}, 1};
  int32_t* all = tables;
  int32_t* grp[2] = {tables + (nchains + 1), tables + 2 * (nchains + 1)};
  int32_t acc = 0, accg[2] = {0, 0};
  // A^(1) staging need and LDS group (light / heavy: one inner launch each)
  // of a chain; one inner pass stages at most 64 rank columns
  auto need_of = [&](const ChainDesc& d) {
    const size_t rt16 = std::min<size_t>(16 * (size_t)((d.R + 15) / 16), 64);
    const size_t need32 = sizeof(float) * rt16 * fit_a0_stride(d.dims[0]);
    const size_t need16 = 2 * sizeof(uint16_t) * rt16 * fit_a0_stride16(d.dims[0]);
    size_t need = (d.dtype == CPD_BF16 && need16 <= kFitLdsMax) ? need16 : need32;
    if (need > kFitLdsMax) need = 0;  // A^(1) read from global memory
    return need;
  };
  auto rows_of = [&](const ChainDesc& d) {
    int64_t J0 = 1;
    for (int k = 1; k < d.N; ++k) J0 *= d.dims[k];
    return J0;
  };
  // rows per block of a chain: at least kFitRowsMin (each block stages
  // A^(1), and the members of a full batch or server round share the GPU, so
  // more, shorter blocks only add staging), more for tensors that would
  // otherwise take over kFitBlocksMax blocks (two per CU).  A function of
  // the chain alone: a batch member and a single handle on the same tensor
  // split their rows the same way, so their fits agree to the bit.
  auto rpb_of = [&](int64_t J0) {
    const int64_t r = (J0 + kFitBlocksMax - 1) / kFitBlocksMax;
    return r < kFitRowsMin ? (int64_t)kFitRowsMin : r;
  };
  for (int c = 0; c < nchains; ++c) {
    const ChainDesc& d = descs[c];
    all[c] = acc;
    grp[0][c] = accg[0];
    grp[1][c] = accg[1];
    if (d.R > 64) fp.passes = 2;
    const size_t need = need_of(d);
    const int g = need <= kFitLightLds ? 0 : 1;
    const int64_t J0 = rows_of(d), rpb = rpb_of(J0);
    int64_t nb = (J0 + rpb - 1) / rpb;
    if (nb < 1) nb = 1;
    if (nb > kFitParts) nb = kFitParts;
    acc += (int32_t)nb;
    accg[g] += (int32_t)nb;
    if (need > fp.lds[g]) fp.lds[g] = need;
  }
  all[nchains] = acc;
  grp[0][nchains] = accg[0];
  grp[1][nchains] = accg[1];
  fp.blocks[0] = accg[0];
  fp.blocks[1] = accg[1];
  return fp;
}

hipError_t launch_fit(const ChainDesc* d_descs, const int32_t* d_tables, int nchains,
                      const FitPlan& fp, int dtype, bool inner, hipStream_t stream) {
  static std::atomic<uint32_t> attr_f32{0}, attr_bf16{0};
  hipError_t ea = set_lds_limit_once((const void*)fit_partial_kernel<float, true>,
                                     (int)kFitLdsMax, &attr_f32);
  if (ea != hipSuccess) return ea;
  ea = set_lds_limit_once((const void*)fit_partial_kernel<uint16_t, true>, (int)kFitLdsMax,
                          &attr_bf16);
  if (ea != hipSuccess) return ea;
  for (int pass = 0; pass < (inner ? fp.passes : 1); ++pass) {
    const int r_off = 64 * pass;
    for (int g = 0; g < 2; ++g) {
      if (fp.blocks[g] == 0) continue;
      const int32_t* tab = d_tables + (g + 1) * (nchains + 1);
      const dim3 grid((unsigned)fp.blocks[g]);
      const size_t lds = inner ? fp.lds[g] : 0;
      const int lds_floats = (int)(lds / sizeof(float));
      if (dtype == CPD_BF16) {
        if (inner)
          hipLaunchKernelGGL((fit_partial_kernel<uint16_t, true>), grid, dim3(kFitBlock), lds,
                             stream, d_descs, tab, nchains, lds_floats, r_off);
        else
          hipLaunchKernelGGL((fit_partial_kernel<uint16_t, false>), grid, dim3(kFitBlock), 0,
                             stream, d_descs, tab, nchains, 0, 0);
      } else {
        if (inner)
          hipLaunchKernelGGL((fit_partial_kernel<float, true>), grid, dim3(kFitBlock), lds,
                             stream, d_descs, tab, nchains, lds_floats, r_off);
        else
          hipLaunchKernelGGL((fit_partial_kernel<float, false>), grid, dim3(kFitBlock), 0, stream,
                             d_descs, tab, nchains, 0, 0);
      }
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  if (inner)
    hipLaunchKernelGGL((fit_final_kernel<true>), dim3(nchains), dim3(1024), 0, stream, d_descs,
                       d_tables);
  else
    hipLaunchKernelGGL((fit_final_kernel<false>), dim3(nchains), dim3(1024), 0, stream, d_descs,
                       d_tables);
  return hipGetLastError();
}

}  // namespace cpdmi
