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
// One pass over copy n (row j = fibre j) and two small kernels:
//   variance_pass_kernel<RT>  blocks of 16-row tiles of a row range and a
//                             group of 16-column tiles: the KRP rows z_j of
//                             the tile (LDS), then per column tile on the
//                             matrix cores both A^(n) z_j (Z tile as the A
//                             operand, A^(n) rows from LDS as the B operand)
//                             minus x_j, squared and summed per row, and the
//                             block's part of M = X_(n) Z^(n) (Z^T as the A
//                             operand, the same fibre values as the B
//                             operand).  The row sums of the group's columns
//                             times ||z_j||^2 / p_j are summed over the
//                             block's rows into one FP64 term per block (the
//                             sum over column groups distributes over the
//                             product), so nothing of size J is stored;
//   variance_msum_kernel      M: the block parts summed in a fixed order
//                             (FP64);
//   variance_final_kernel     the block terms summed in a fixed order, the
//                             Gram Hadamard product, grad f and the variance.
//
// Scratch (caller-owned, or the library's static array for the variant that
// allocates nothing): the descriptor copy, a state, the sampler's CDFs, the
// blocks' FP32 parts of M, M in FP64, the block terms and the result.
#include <cstring>
#include <mutex>
#include <string>

#include "cpd_runtime.hpp"

namespace cpdmi {

typedef float vf4 __attribute__((ext_vector_type(4)));


constexpr int kVpThreads = 256;  // threads of a pass block (four waves)

// Column tiles of one wave held in registers for a rank-tile count RT.
__host__ __device__ constexpr int var_tiles_per_wave(int rt) { return rt == 1 ? 5 : (rt == 2 ? 4 : 2); }

// LDS of a pass block: A^(n) rows of the group's columns (ranks padded to
// 16 RT), two Z tiles (16 rows, stride 16 RT + 1) and the row multi-indices
// of two tiles (the current one and the next), the per-wave row sums and the
// rows' ||z_j||^2 / p_j.
__host__ __device__ inline size_t var_pass_lds(int tpg, int RT) {
  return sizeof(float) * (size_t)tpg * 16 * 16 * RT + 2 * sizeof(float) * 16 * (16 * RT + 1) +
         2 * sizeof(int32_t) * 16 * kMaxModes + sizeof(double) * 5 * 16;
}

// Block (c, g): rows [c rpc, (c + 1) rpc) in 16-row tiles, column tiles
// [g tpg, (g + 1) tpg); wave w takes column tiles g tpg + w, + 4, ...
//   terms[c * ngroups + g]  sum over the block's rows j of
//                           (sum over the group's columns of (A^(n) z_j - x_j)^2)
//                           * ||z_j||^2 / p_j   (FP64)
//   part[c][i][r]           sum over the block's rows of x_j(i) z_j(r)
template <int RT>
__global__ void __launch_bounds__(kVpThreads) variance_pass_kernel(
    const ChainDesc* __restrict__ dp, int n, int64_t rpc, int tpg, float* __restrict__ part,
    double* __restrict__ terms) {
  extern __shared__ __align__(16) unsigned char vsm[];
  constexpr int Rp = 16 * RT, ZS = Rp + 1, MT = var_tiles_per_wave(RT);
  const int In = dp->dims[n], R = dp->R, N = dp->N;
  int64_t J = 1;
  for (int k = 0; k < N; ++k)
    if (k != n) J *= dp->dims[k];
  const int c = blockIdx.x, g = blockIdx.y;
  const int nct = (In + 15) / 16;
  const int ct0 = g * tpg, ct1 = ct0 + tpg < nct ? ct0 + tpg : nct;
  const int64_t r0 = (int64_t)c * rpc, r1 = r0 + rpc < J ? r0 + rpc : J;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int gl = lane >> 4, cl = lane & 15;
  float* As = (float*)vsm;                                // [tpg * 16][Rp]
  float* Zb = As + (size_t)tpg * 16 * Rp;                 // [2][16][ZS]
  int32_t* ikb = (int32_t*)(Zb + 2 * 16 * ZS);            // [2][16][kMaxModes]
  double* red = (double*)(vsm + var_pass_lds(tpg, RT) - sizeof(double) * 5 * 16);  // [4][16]
  double* zwl = red + 4 * 16;                             // ||z_j||^2 / p_j of the tile's rows
  double tacc = 0.0;                                      // threads 0..15: their rows' terms
  const CPD_GLOBAL float* An = gmem((const float*)dp->A[n]);
  for (int e = tid; e < tpg * 16 * Rp; e += kVpThreads) {
    const int i = ct0 * 16 + e / Rp, r = e % Rp;
    As[e] = (i < In && r < R) ? An[(int64_t)i * R + r] : 0.f;
  }
  // row multi-index of row r0 + tid (threads 0..15), advanced by 16 per tile
  // (odometer over the modes k != n, the lowest fastest)
  int ik[kMaxModes];
  auto advance = [&]() {
    int carry = 16;
    for (int k = 0; k < N && carry; ++k) {
      if (k == n) continue;
      const int v = ik[k] + carry;
      carry = v / dp->dims[k];
      ik[k] = v - carry * dp->dims[k];
    }
  };
  if (tid < 16) {
    int64_t rem = r0 + tid;
    for (int k = 0; k < N; ++k) {
      ik[k] = 0;
      if (k == n) continue;
      const int64_t nx = rem / dp->dims[k];
      ik[k] = (int)(rem - nx * dp->dims[k]);
      rem = nx;
    }
    for (int k = 0; k < N; ++k) ikb[tid * kMaxModes + k] = ik[k];
    advance();
    for (int k = 0; k < N; ++k) ikb[(16 + tid) * kMaxModes + k] = ik[k];
    advance();
  }
  __syncthreads();
  // z_j(r) = prod_{k != n} A^(k)(i_k, r), ascending k, for entry e of the
  // tile starting at row tb whose indices are in buffer ib
  constexpr int ZE = (16 * Rp + kVpThreads - 1) / kVpThreads;  // entries per thread
  auto z_tile = [&](int64_t tb, int ib, float (&zv)[ZE]) {
#pragma unroll
    for (int u = 0; u < ZE; ++u) {
      const int e = tid + u * kVpThreads;
      const int row = e / Rp, r = e - row * Rp;
      float z = 0.f;
      if (e < 16 * Rp && tb + row < r1 && r < R) {
        bool first = true;
        for (int k = 0; k < N; ++k) {
          if (k == n) continue;
          const float a = gmem((const float*)dp->A[k])
              [(int64_t)ikb[(ib * 16 + row) * kMaxModes + k] * R + r];
          z = first ? a : z * a;
          first = false;
        }
      }
      zv[u] = z;
    }
  };
  auto z_store = [&](int zbuf, const float (&zv)[ZE]) {
#pragma unroll
    for (int u = 0; u < ZE; ++u) {
      const int e = tid + u * kVpThreads;
      if (e < 16 * Rp) Zb[(zbuf * 16 + e / Rp) * ZS + e % Rp] = zv[u];
    }
  };
  {
    float zv[ZE];
    z_tile(r0, 0, zv);
    z_store(0, zv);
  }
  __syncthreads();
  vf4 macc[MT][RT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) macc[m][rt] = vf4{0.f, 0.f, 0.f, 0.f};
  const int64_t ld = dp->ld[n];
  int cur = 0;
  for (int64_t t0 = r0; t0 < r1; t0 += 16, cur ^= 1) {
    const float* Zt = Zb + cur * 16 * ZS;
    // in flight together: this tile's fibre values, the next tile's factor
    // rows, this tile's CDF entries
    float xs[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int ct = ct0 + wave + 4 * m;
      const int i = ct * 16 + cl;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t j = t0 + 4 * gl + q;
        float v = 0.f;
        if (ct < ct1 && j < r1 && i < In) {
          if (dp->dtype == CPD_BF16)
            v = __uint_as_float((uint32_t)gmem((const uint16_t*)dp->X[n])[j * ld + i] << 16);
          else
            v = gmem((const float*)dp->X[n])[j * ld + i];
        }
        xs[m][q] = v;
      }
    }
    float zn[ZE];
    z_tile(t0 + 16, cur ^ 1, zn);
    if (tid < 16) {
      // p_j: product over k != n of q / Q of the sampler's integer CDFs
      double zwv = 0.0;
      if (t0 + tid < r1) {
        double p = 1.0;
        for (int k = 0; k < N; ++k) {
          if (k == n) continue;
          const CPD_GLOBAL double* C = gmem((const double*)dp->C[k]);
          const int i = ikb[(cur * 16 + tid) * kMaxModes + k];
          const double Q = C[dp->dims[k] - 1];
          p = p * ((C[i] - (i ? C[i - 1] : 0.0)) / Q);
        }
        float z2 = 0.f;
        for (int r = 0; r < Rp; ++r) z2 = fmaf(Zt[tid * ZS + r], Zt[tid * ZS + r], z2);
        zwv = p > 0.0 ? (double)z2 / p : 0.0;
      }
      zwl[tid] = zwv;
    }
    double r2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int ct = ct0 + wave + 4 * m;
      if (ct >= ct1) break;
      const int i = ct * 16 + cl;
      const float* x = xs[m];
      // A^(n) z_j for rows 4 gl + q, column i: K = rank
      vf4 y = vf4{0.f, 0.f, 0.f, 0.f};
      const float* Ar = As + (size_t)((ct - ct0) * 16 + cl) * Rp;
#pragma unroll
      for (int s = 0; s < 4 * RT; ++s)
        y = __builtin_amdgcn_mfma_f32_16x16x4f32(Zt[cl * ZS + 4 * s + gl], Ar[4 * s + gl], y, 0,
                                                 0, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float d = y[q] - x[q];
        if (t0 + 4 * gl + q < r1 && i < In) r2[q] += (double)(d * d);
      }
      // M^T tile += Z^T X: K-step q holds rows 4 gl + q
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          macc[m][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(Zt[(4 * gl + q) * ZS + rt * 16 + cl],
                                                             x[q], macc[m][rt], 0, 0, 0);
    }
    // the next tile's Z; the indices of the tile after it replace this tile's
    z_store(cur ^ 1, zn);
    if (tid < 16) {
      for (int k = 0; k < N; ++k) ikb[(cur * 16 + tid) * kMaxModes + k] = ik[k];
      advance();
    }
    // per-row sums over the columns: the 16 lanes of a group, then the waves
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) r2[q] += __shfl_xor(r2[q], o);
      if (cl == 0) red[wave * 16 + 4 * gl + q] = r2[q];
    }
    __syncthreads();
    if (tid < 16 && t0 + tid < r1)
      tacc += (red[tid] + red[16 + tid] + red[32 + tid] + red[48 + tid]) * zwl[tid];
    __syncthreads();
  }
  // the block's term: the 16 row-slot sums in order
  if (tid < 16) red[tid] = tacc;
  __syncthreads();
  if (tid == 0) {
    double tsum = 0.0;
    for (int q = 0; q < 16; ++q) tsum += red[q];
    terms[(int64_t)c * gridDim.y + g] = tsum;
  }
  // the block's part of M: macc[m][rt][q] = M^T(rank 16 rt + 4 gl + q, column ct * 16 + cl)
  float* out = part + (int64_t)c * In * R;
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int ct = ct0 + wave + 4 * m;
    if (ct >= ct1) break;
    const int i = ct * 16 + cl;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * rt + 4 * gl + q;
        if (r < R && i < In) out[(int64_t)i * R + r] = macc[m][rt][q];
      }
  }
}

// M(e) = sum over the parts, in a fixed order (FP64): 16 entries per block,
// 64 lane groups of 16 lanes summing parts g, g + 64, ..., then the groups
// in order.
__global__ void __launch_bounds__(1024) variance_msum_kernel(const float* __restrict__ part,
                                                             int nparts, int E,
                                                             double* __restrict__ M) {
  __shared__ double red[64][17];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = wave * 4 + (lane >> 4), ec = lane & 15;
  const int e = blockIdx.x * 16 + ec;
  double s = 0.0;
  if (e < E)
    for (int b = grp; b < nparts; b += 64) s += (double)gmem(part)[(int64_t)b * E + e];
  red[grp][ec] = s;
  __syncthreads();
  if (threadIdx.x < 16 && blockIdx.x * 16 + (int)threadIdx.x < E) {
    double m = 0.0;
    for (int q = 0; q < 64; ++q) m += red[q][threadIdx.x];
    M[blockIdx.x * 16 + threadIdx.x] = m;
  }
}

// out[0] = variance, out[1] = (1/B) sum of the terms, out[2] = ||grad f||^2 / B.
__global__ void __launch_bounds__(1024) variance_final_kernel(const ChainDesc* __restrict__ dp,
                                                              int n, const double* __restrict__ M,
                                                              int nblocks,
                                                              const double* __restrict__ terms,
                                                              double* __restrict__ out) {
  __shared__ double red[16];
  constexpr int kVr = 16 * kMaxRankTiles;  // the variance takes R <= 64
  __shared__ double had[kVr * kVr];
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
  // H = hadamard_{k != n} A^(k)T A^(k), FP64: every thread takes one (pair,
  // row range) item; the row ranges of a pair are summed in a fixed order
  // items: npairs * nrg <= max(npairs, blockDim.x) <= kVr (kVr + 1) / 2
  __shared__ double gpart[kVr * (kVr + 1) / 2];
  for (int p = tid; p < R2; p += blockDim.x) had[p] = 1.0;
  const int npairs = R * (R + 1) / 2;
  for (int k = 0; k < dp->N; ++k) {
    if (k == n) continue;
    const CPD_GLOBAL float* A = gmem((const float*)dp->A[k]);
    const int Ik = dp->dims[k];
    int nrg = (int)blockDim.x / npairs;
    if (nrg < 1) nrg = 1;
    if (nrg > Ik) nrg = Ik;
    __syncthreads();
    for (int it = tid; it < npairs * nrg; it += blockDim.x) {
      const int pr = it % npairs, rg = it / npairs;
      int r = 0, rem = pr;
      while (rem >= R - r) {
        rem -= R - r;
        ++r;
      }
      const int cidx = r + rem;
      const int i0 = (int)((int64_t)rg * Ik / nrg), i1 = (int)((int64_t)(rg + 1) * Ik / nrg);
      double acc = 0.0;
      for (int i = i0; i < i1; ++i)
        acc += (double)A[(int64_t)i * R + r] * (double)A[(int64_t)i * R + cidx];
      gpart[it] = acc;
    }
    __syncthreads();
    for (int pr = tid; pr < npairs; pr += blockDim.x) {
      int r = 0, rem = pr;
      while (rem >= R - r) {
        rem -= R - r;
        ++r;
      }
      const int cidx = r + rem;
      double gsum2 = 0.0;
      for (int rg = 0; rg < nrg; ++rg) gsum2 += gpart[rg * npairs + pr];
      had[r * R + cidx] *= gsum2;
      if (cidx != r) had[cidx * R + r] *= gsum2;
    }
  }
  __syncthreads();
  // grad f = A^(n) H - M
  const CPD_GLOBAL float* An = gmem((const float*)dp->A[n]);
  double gsum = 0.0;
  for (int e = tid; e < In * R; e += blockDim.x) {
    const int i = e / R, r = e - i * R;
    const double m = M[e];
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

// Scratch layout and launch shape of one variance evaluation.
struct VarPlan {
  int ngroups, tpg, nchunks;
  int64_t J, rpc;
  size_t lds;
  size_t desc, state, cdf, part, M, terms, out, total;
};

// Bytes of the blocks' FP32 parts of M, at most: the number of row chunks
// is capped so that nchunks * I_n * R * 4 stays within this.
constexpr size_t kVarPartBudget = 16u << 20;
// Row chunks of the pass planned by variance_scratch_bytes: at least as many
// pass blocks as any MI355X holds at once (256 CUs x 4 blocks).
constexpr int kVarMaxBlocks = 1024;

// target_blocks: pass blocks the GPU holds at once (one round of blocks
// measured fastest: 66 vs 90 us at 300^3 against 1.2 rounds).
static VarPlan plan_variance(const ChainDesc& d, int n, int target_blocks) {
  VarPlan v;
  v.J = 1;
  for (int k = 0; k < d.N; ++k)
    if (k != n) v.J *= d.dims[k];
  const int RT = (d.R + 15) / 16;
  const int nct = (d.dims[n] + 15) / 16;
  const int tmax = 4 * var_tiles_per_wave(RT);  // column tiles of one block
  v.ngroups = (nct + tmax - 1) / tmax;
  v.tpg = (nct + v.ngroups - 1) / v.ngroups;
  v.lds = var_pass_lds(v.tpg, RT);
  // one round of resident blocks, rows in whole 16-row tiles
  int64_t nch = (target_blocks + v.ngroups - 1) / v.ngroups;
  const int64_t cap = (int64_t)(kVarPartBudget / ((size_t)d.dims[n] * d.R * sizeof(float)));
  if (nch > cap) nch = cap;
  if (nch < 1) nch = 1;
  const int64_t tiles = (v.J + 15) / 16;
  if (nch > tiles) nch = tiles;
  v.rpc = (tiles + nch - 1) / nch * 16;
  v.nchunks = (int)((v.J + v.rpc - 1) / v.rpc);
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
  v.part = take(sizeof(float) * (size_t)v.nchunks * d.dims[n] * d.R);
  v.M = take(sizeof(double) * (size_t)d.dims[n] * d.R);
  v.terms = take(sizeof(double) * (size_t)v.nchunks * v.ngroups);
  v.out = take(sizeof(double) * 4);
  v.total = off;
  return v;
}

template <int RT>
static hipError_t launch_pass(const VarPlan& v, const ChainDesc* dd, int n, char* base,
                              hipStream_t stream) {
  static std::atomic<uint32_t> attr{0};
  hipError_t e = set_lds_limit_once((const void*)variance_pass_kernel<RT>, 160 * 1024, &attr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((variance_pass_kernel<RT>), dim3(v.nchunks, v.ngroups), dim3(kVpThreads),
                     v.lds, stream, dd, n, v.rpc, v.tpg, (float*)(base + v.part),
                     (double*)(base + v.terms));
  return hipGetLastError();
}

// Pass blocks resident on the whole device at once for an LDS size.
template <int RT>
static int pass_capacity(size_t lds) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, variance_pass_kernel<RT>, kVpThreads,
                                                   lds) != hipSuccess ||
      cus <= 0 || per_cu <= 0)
    return 768;
  return cus * per_cu;
}

size_t variance_scratch_bytes(const ChainDesc& hd, int n) {
  return plan_variance(hd, n, kVarMaxBlocks).total;
}

// Scratch of the variance evaluation that allocates nothing
// (cpd_variance_noalloc): one array per device, held until the process
// ends.  Its size covers every problem within the library's limits: the
// parts of M are capped at kVarPartBudget, M itself takes at most
// CPD_MAX_DIM * 64 doubles (the variance takes R <= 64), the CDFs CPD_MAX_MODES * CPD_MAX_DIM
// doubles, the rest a few KiB.  In host code the array's name is only a
// host-side stand-in; kernels and copies use the device address returned by
// hipGetSymbolAddress for the current device.
static __device__ __align__(256) char scratch[kVarStaticScratch];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];  // per device ordinal; null until looked up

cpd_status variance_static_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) {
    set_error("device ordinal beyond the static scratch table");
    return CPD_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(variance scratch)");
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return CPD_OK;
}

cpd_status variance_eval(const ChainDesc& hd, size_t lds, size_t grid_refresh_lds, int n,
                         int sampler, hipStream_t stream, double* out3, void* scratch_v,
                         size_t scratch_bytes) {
  VarPlan v = plan_variance(hd, n, 768);
  int cap = 768;
  switch (hd.RT) {
    case 1: cap = pass_capacity<1>(v.lds); break;
    case 2: cap = pass_capacity<2>(v.lds); break;
    case 3: cap = pass_capacity<3>(v.lds); break;
    default: cap = pass_capacity<4>(v.lds); break;
  }
  v = plan_variance(hd, n, cap < kVarMaxBlocks ? cap : kVarMaxBlocks);
  if (!scratch_v || v.total > scratch_bytes) {
    set_error("variance scratch of " + std::to_string(scratch_bytes) + " bytes; this mode needs " +
              std::to_string(v.total));
    return CPD_E_OOM;
  }
  char* base = (char*)scratch_v;
  // the requested sampler's distributions of the current factors
  ChainDesc d = hd;
  d.sampler = sampler;
  size_t coff = 0;
  for (int k = 0; k < d.N; ++k) {
    d.C[k] = (double*)(base + v.cdf) + coff;
    coff += d.dims[k];
  }
  d.state = (ChainState*)(base + v.state);
  d.active = 1;
  d.autostop = 0;
  ChainDesc* dd = (ChainDesc*)(base + v.desc);
  // the state starts at zero (status, clock); every other region is
  // written in full before it is read
  const ChainState zero_state{};
  hipError_t e = hipMemcpyAsync(dd, &d, sizeof d, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + v.state, &zero_state, sizeof zero_state, hipMemcpyHostToDevice,
                       stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(desc)");
  if (grid_refresh_lds > 0) {
    e = launch_wide_refresh(dd, d.RT, grid_refresh_lds, nullptr, -1, d.N, stream);
  } else {
    StepArgs a{};
    a.op = OP_REFRESH;
    e = launch_chain_kernel(dd, 1, d.RT, lds, a, stream);
  }
  if (e != hipSuccess) return hip_fail(e, "refresh kernel");
  switch (d.RT) {
    case 1: e = launch_pass<1>(v, dd, n, base, stream); break;
    case 2: e = launch_pass<2>(v, dd, n, base, stream); break;
    case 3: e = launch_pass<3>(v, dd, n, base, stream); break;
    default: e = launch_pass<4>(v, dd, n, base, stream); break;
  }
  if (e != hipSuccess) return hip_fail(e, "variance pass kernel");
  const int E = d.dims[n] * d.R;
  hipLaunchKernelGGL(variance_msum_kernel, dim3((E + 15) / 16), dim3(1024), 0, stream,
                     (const float*)(base + v.part), v.nchunks, E, (double*)(base + v.M));
  hipLaunchKernelGGL(variance_final_kernel, dim3(1), dim3(1024), 0, stream, dd, n,
                     (const double*)(base + v.M), v.nchunks * v.ngroups,
                     (const double*)(base + v.terms), (double*)(base + v.out));
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "variance kernels");
  ChainState st;
  e = hipMemcpyAsync(&st, base + v.state, sizeof st, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out3, base + v.out, sizeof(double) * 3, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "variance result");
  if (st.status != 0) {
    describe_status(st.status);
    return st.status;
  }
  return CPD_OK;
}

}  // namespace cpdmi
