// Exact variance of the sampled gradient of one mode (Section 4, the
// variance theorem and Table 1), at the current factors:
//
//   E ||G - grad f||_F^2 = (1/B) ( sum_j ||r_j||^2 ||z_j||^2 / p_j - ||grad f||_F^2 )
//
// with z_j the KRP row j of Z^(n), r_j = A^(n) z_j - x_j the residual of
// fibre j, p_j the probability the sampler gives row j (product of the
// per-mode q/Q of the integer CDFs), and grad f = A^(n) (hadamard_{k!=n}
// A^(k)T A^(k)) - X_(n) Z^(n).
//
// Three kernels over copy n (row j = fibre j):
//   variance_mttkrp_kernel  partial sums of M = X_(n) Z^(n): one wave per
//                           (16-column tile of I_n, range of rows), M^T
//                           tiles on the matrix cores (Z^T as the A operand,
//                           the fibres as the B operand);
//   variance_terms_kernel   per 16-row tile: A^(n) z_j for 16 columns at a
//                           time on the matrix cores (Z tile as the A
//                           operand, A^(n)^T as the B operand), minus x_j,
//                           squared and summed per row; then
//                           ||r_j||^2 ||z_j||^2 / p_j summed in FP64;
//   variance_final_kernel   sum of the partials in a fixed order, the Gram
//                           Hadamard product, grad f and the variance (FP64).
#include <cstring>
#include <string>

#include "cpd_runtime.hpp"

namespace cpdmi {

typedef float vf4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kVarWaveRows = 16;

// Element e of copy n (row j, column i) as FP32.
__device__ __forceinline__ float load_x(const ChainDesc* dp, int n, int64_t j, int i) {
  const int64_t off = j * dp->ld[n] + i;
  if (dp->dtype == CPD_BF16) {
    const uint16_t v = gmem((const uint16_t*)dp->X[n])[off];
    return __uint_as_float((uint32_t)v << 16);
  }
  return gmem((const float*)dp->X[n])[off];
}

// Multi-index of row j of copy n over the modes k != n (ascending, the
// lowest fastest): writes i_k into ik[k].
__device__ __forceinline__ void row_index(const ChainDesc* dp, int n, int64_t j, int* ik) {
  int64_t rem = j;
  for (int k = 0; k < dp->N; ++k) {
    if (k == n) continue;
    const int Ik = dp->dims[k];
    const int64_t nx = rem / Ik;
    ik[k] = (int)(rem - nx * Ik);
    rem = nx;
  }
}

// z_j(r) = prod_{k != n} A^(k)(i_k, r) (ascending k); 0 for r >= R.
__device__ __forceinline__ float z_entry(const ChainDesc* dp, int n, const int* ik, int r) {
  if (r >= dp->R) return 0.f;
  float z = 1.f;
  bool first = true;
  for (int k = 0; k < dp->N; ++k) {
    if (k == n) continue;
    const float a = gmem((const float*)dp->A[k])[(int64_t)ik[k] * dp->R + r];
    z = first ? a : z * a;
    first = false;
  }
  return z;
}

}  // namespace

// One wave per block.  Block (t, c): column tile t (16 columns of I_n),
// rows [c * rpc, (c + 1) * rpc).  partial[c][i][r] = sum over its rows of
// x_j(i) z_j(r).
__global__ void __launch_bounds__(64) variance_mttkrp_kernel(const ChainDesc* __restrict__ dp,
                                                             int n, int nchunks,
                                                             float* __restrict__ partial) {
  const int In = dp->dims[n], R = dp->R, RT = (R + 15) / 16;
  int64_t J = 1;
  for (int k = 0; k < dp->N; ++k)
    if (k != n) J *= dp->dims[k];
  const int ntiles = (In + 15) / 16;
  const int tile = blockIdx.x % ntiles, c = blockIdx.x / ntiles;
  const int64_t rpc = (J + nchunks - 1) / nchunks;
  const int64_t j0 = (int64_t)c * rpc, j1 = j0 + rpc < J ? j0 + rpc : J;
  const int lane = threadIdx.x, kg = lane >> 4, rq = lane & 15;
  const int i = tile * 16 + rq;
  vf4 acc[4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) acc[rt] = vf4{0.f, 0.f, 0.f, 0.f};
  int ik[kMaxModes];
  for (int64_t jb = j0; jb < j1; jb += 4) {
    const int64_t j = jb + kg;
    const bool ok = j < j1;
    float x = 0.f;
    float zr[4] = {0.f, 0.f, 0.f, 0.f};
    if (ok) {
      if (i < In) x = load_x(dp, n, j, i);
      row_index(dp, n, j, ik);
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
        if (rt < RT) zr[rt] = z_entry(dp, n, ik, 16 * rt + rq);
    }
    // A operand: Z^T[rank 16 rt + rq][row slot kg]; B operand: X[row slot kg][column rq]
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
      if (rt < RT) acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(zr[rt], x, acc[rt], 0, 0, 0);
  }
  // acc[rt][q] = M^T(rank 16 rt + 4 kg + q, column rq of the tile)
  float* out = partial + (int64_t)c * In * R;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
    if (rt < RT)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * rt + 4 * kg + q;
        if (r < R && i < In) out[(int64_t)i * R + r] = acc[rt][q];
      }
}

// One wave per block, rows [b * rpb, (b + 1) * rpb) in 16-row tiles.
// terms[b] = sum over its rows of ||r_j||^2 ||z_j||^2 / p_j (FP64).
__global__ void __launch_bounds__(64) variance_terms_kernel(const ChainDesc* __restrict__ dp,
                                                            int n, int nblocks,
                                                            double* __restrict__ terms) {
  const int In = dp->dims[n], R = dp->R, RT = (R + 15) / 16;
  int64_t J = 1;
  for (int k = 0; k < dp->N; ++k)
    if (k != n) J *= dp->dims[k];
  const int64_t rpb = ((J + nblocks - 1) / nblocks + 15) / 16 * 16;
  const int64_t r0 = (int64_t)blockIdx.x * rpb, r1 = r0 + rpb < J ? r0 + rpb : J;
  const int lane = threadIdx.x, kg = lane >> 4, rq = lane & 15;
  const CPD_GLOBAL float* An = gmem((const float*)dp->A[n]);
  double total = 0.0;
  int ik[kMaxModes];
  for (int64_t t0 = r0; t0 < r1; t0 += 16) {
    // this lane's A-operand row and its z entries at ranks 4 s + kg
    const int64_t ja = t0 + rq;
    const bool oka = ja < r1;
    float za[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) za[s] = 0.f;
    double zp = 0.0;  // ||z||^2 / p of row ja (complete after the reduction)
    double p = 1.0;
    if (oka) {
      row_index(dp, n, ja, ik);
#pragma unroll
      for (int s = 0; s < 16; ++s)
        if (s < 4 * RT) za[s] = z_entry(dp, n, ik, 4 * s + kg);
      for (int k = 0; k < dp->N; ++k) {
        if (k == n) continue;
        const CPD_GLOBAL double* C = gmem((const double*)dp->C[k]);
        const double Q = C[dp->dims[k] - 1];
        const double lo = ik[k] ? C[ik[k] - 1] : 0.0;
        p = p * ((C[ik[k]] - lo) / Q);
      }
    }
    float z2 = 0.f;
#pragma unroll
    for (int s = 0; s < 16; ++s) z2 = fmaf(za[s], za[s], z2);
    double z2d = (double)z2;
    z2d += __shfl_xor(z2d, 16);
    z2d += __shfl_xor(z2d, 32);
    zp = (oka && p > 0.0) ? z2d / p : 0.0;
    // residual rows 4 kg + q of the tile, 16 columns at a time
    double r2[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i0 = 0; i0 < In; i0 += 16) {
      const int i = i0 + rq;
      vf4 acc = vf4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        if (s < 4 * RT) {
          const int r = 4 * s + kg;
          const float b = (i < In && r < R) ? An[(int64_t)i * R + r] : 0.f;
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(za[s], b, acc, 0, 0, 0);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t j = t0 + 4 * kg + q;
        if (j < r1 && i < In) {
          const float d = acc[q] - load_x(dp, n, j, i);
          r2[q] += (double)(d * d);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) r2[q] += __shfl_xor(r2[q], o);
      // z^2/p of row 4 kg + q sits in lane (kg' = 0, rq = 4 kg + q)
      const double zpq = __shfl(zp, 4 * kg + q);
      if (rq == 0 && t0 + 4 * kg + q < r1) total += r2[q] * zpq;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) total += __shfl_xor(total, o);
  if (lane == 0) terms[blockIdx.x] = total;
}

// out[0] = variance, out[1] = (1/B) sum of the terms, out[2] = ||grad f||^2 / B.
__global__ void __launch_bounds__(1024) variance_final_kernel(const ChainDesc* __restrict__ dp,
                                                              int n, int nchunks,
                                                              const float* __restrict__ partial,
                                                              int nblocks,
                                                              const double* __restrict__ terms,
                                                              double* __restrict__ out) {
  __shared__ double red[16];
  __shared__ double had[kMaxRank * kMaxRank];
  __shared__ float rows[64 * kMaxRank];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R = dp->R, R2 = R * R, In = dp->dims[n];
  double t = 0.0;
  for (int b = tid; b < nblocks; b += blockDim.x) t += terms[b];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
  if (lane == 0) red[wave] = t;
  __syncthreads();
  double T = 0.0;
  for (int w = 0; w < 16; ++w) T += red[w];
  __syncthreads();
  // H = hadamard_{k != n} A^(k)T A^(k), FP64, rows staged through LDS
  for (int p = tid; p < R2; p += blockDim.x) had[p] = 1.0;
  for (int k = 0; k < dp->N; ++k) {
    if (k == n) continue;
    const CPD_GLOBAL float* A = gmem((const float*)dp->A[k]);
    const int Ik = dp->dims[k];
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i0 = 0; i0 < Ik; i0 += 64) {
      const int nr = Ik - i0 < 64 ? Ik - i0 : 64;
      __syncthreads();
      for (int e = tid; e < nr * R; e += blockDim.x) rows[e] = A[(int64_t)i0 * R + e];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int p = tid + q * 1024;
        if (p < R2) {
          const int r = p / R, c = p - r * R;
          for (int i = 0; i < nr; ++i) g[q] += (double)rows[i * R + r] * (double)rows[i * R + c];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (tid + q * 1024 < R2) had[tid + q * 1024] *= g[q];
    __syncthreads();
  }
  // grad f = A^(n) H - M, M = sum of the partial MTTKRPs (fixed order)
  const CPD_GLOBAL float* An = gmem((const float*)dp->A[n]);
  double gsum = 0.0;
  for (int e = tid; e < In * R; e += blockDim.x) {
    const int i = e / R, r = e - i * R;
    double m = 0.0;
    for (int c = 0; c < nchunks; ++c) m += (double)partial[(int64_t)c * In * R + e];
    double ah = 0.0;
    for (int s = 0; s < R; ++s) ah += (double)An[(int64_t)i * R + s] * had[s * R + r];
    const double gr = ah - m;
    gsum += gr * gr;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) gsum += __shfl_xor(gsum, o);
  if (lane == 0) red[wave] = gsum;
  __syncthreads();
  if (tid == 0) {
    double G2 = 0.0;
    for (int w = 0; w < 16; ++w) G2 += red[w];
    const double B = (double)dp->B;
    out[0] = (T - G2) / B;
    out[1] = T / B;
    out[2] = G2 / B;
  }
}

// Scratch layout of one variance evaluation.
struct VarPlan {
  int nchunks, nblocks;
  size_t desc, state, cdf, partial, terms, out, total;
};

static VarPlan plan_variance(const ChainDesc& d, int n) {
  VarPlan v;
  int64_t J = 1;
  for (int k = 0; k < d.N; ++k)
    if (k != n) J *= d.dims[k];
  const int ntiles = (d.dims[n] + 15) / 16;
  int64_t nch = (2048 + ntiles - 1) / ntiles;
  const int64_t maxch = (J + 63) / 64;
  v.nchunks = (int)(nch < 1 ? 1 : (nch > maxch ? maxch : nch));
  int64_t nb = (J + 255) / 256;
  v.nblocks = (int)(nb < 1 ? 1 : (nb > 4096 ? 4096 : nb));
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += (b + 255) / 256 * 256;
    return o;
  };
  int sumdims = 0;
  for (int k = 0; k < d.N; ++k) sumdims += d.dims[k];
  v.desc = take(sizeof(ChainDesc));
  v.state = take(sizeof(ChainState) + 64);
  v.cdf = take(sizeof(double) * sumdims);
  v.partial = take(sizeof(float) * (size_t)v.nchunks * d.dims[n] * d.R);
  v.terms = take(sizeof(double) * v.nblocks);
  v.out = take(sizeof(double) * 4);
  v.total = off;
  return v;
}

cpd_status variance_eval(const ChainDesc& hd, size_t lds, size_t grid_refresh_lds, int n,
                         int sampler, hipStream_t stream, double* out3) {
  const VarPlan v = plan_variance(hd, n);
  char* scratch = nullptr;
  hipError_t e = hipMalloc((void**)&scratch, v.total);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(variance scratch)");
  auto done = [&](cpd_status s) {
    (void)hipStreamSynchronize(stream);
    (void)hipFree(scratch);
    return s;
  };
  e = hipMemsetAsync(scratch, 0, v.total, stream);
  if (e != hipSuccess) return done(hip_fail(e, "hipMemsetAsync"));
  // the requested sampler's distributions of the current factors
  ChainDesc d = hd;
  d.sampler = sampler;
  size_t coff = 0;
  for (int k = 0; k < d.N; ++k) {
    d.C[k] = (double*)(scratch + v.cdf) + coff;
    coff += d.dims[k];
  }
  d.state = (ChainState*)(scratch + v.state);
  d.active = 1;
  d.autostop = 0;
  ChainDesc* dd = (ChainDesc*)(scratch + v.desc);
  e = hipMemcpyAsync(dd, &d, sizeof d, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return done(hip_fail(e, "hipMemcpyAsync(desc)"));
  if (grid_refresh_lds > 0) {
    e = launch_wide_refresh(dd, d.RT, grid_refresh_lds, nullptr, -1, stream);
  } else {
    StepArgs a{};
    a.op = OP_REFRESH;
    e = launch_chain_kernel(dd, 1, d.RT, lds, a, stream);
  }
  if (e != hipSuccess) return done(hip_fail(e, "refresh kernel"));
  const int ntiles = (d.dims[n] + 15) / 16;
  hipLaunchKernelGGL(variance_mttkrp_kernel, dim3(ntiles * v.nchunks), dim3(64), 0, stream, dd, n,
                     v.nchunks, (float*)(scratch + v.partial));
  hipLaunchKernelGGL(variance_terms_kernel, dim3(v.nblocks), dim3(64), 0, stream, dd, n,
                     v.nblocks, (double*)(scratch + v.terms));
  hipLaunchKernelGGL(variance_final_kernel, dim3(1), dim3(1024), 0, stream, dd, n, v.nchunks,
                     (const float*)(scratch + v.partial), v.nblocks,
                     (const double*)(scratch + v.terms), (double*)(scratch + v.out));
  e = hipGetLastError();
  if (e != hipSuccess) return done(hip_fail(e, "variance kernels"));
  ChainState st;
  e = hipMemcpyAsync(&st, scratch + v.state, sizeof st, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out3, scratch + v.out, sizeof(double) * 3, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return done(hip_fail(e, "variance result"));
  if (st.status != 0) {
    describe_status(st.status);
    return done(st.status);
  }
  return done(CPD_OK);
}

}  // namespace cpdmi
