// Internal definitions shared by the host runtime and the gfx950 kernels of
// libcpdmi: the per-decomposition descriptor read by the kernels, the
// workspace layout, the Philox4x64-10 generator and small device helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <atomic>

#include "../../include/cpd.h"

namespace cpdmi {

constexpr int kMaxModes = CPD_MAX_MODES;
constexpr int kMaxRank = CPD_MAX_RANK;
constexpr int kMaxRankTiles = 4;        // rank tiles (R <= 64) of the persistent step, batches,
                                        // the server, leverage scores and the variance
constexpr int kWideRt = 8;              // the grid step's rank tiles for 4 < ceil(R/16) <= 8
constexpr int kGramParts = 4;           // K-parts of the one-tile leverage Gram (256 doubles each)
constexpr int kBlock = 512;             // threads of the persistent step workgroup
constexpr int kWaves = kBlock / 64;
constexpr int kFitBlock = 512;
constexpr int kFitParts = 4096;         // partial sums of the fit / norm kernels
constexpr size_t kAlign = 256;
constexpr int kLdAlign = 64;            // copy rows padded to 64 elements
constexpr int kChunkSteps = 32;         // MFMA K-steps (4 fibres each) per chunk, for VW = RT = 1
constexpr int kFibrePad = 4 * kChunkSteps;  // sampled fibres padded (zero weight) to full chunks
constexpr int kFibreBufs = 2;           // register buffers of fibre chunks in the contraction
constexpr double kRankTol = 1e-12;      // Cholesky pivot^2 <= tol * diagonal => rank deficient
constexpr size_t kLdsBudget = 160 * 1024;  // LDS per workgroup on gfx950
constexpr int kFitRowsMin = 256;        // rows of copy 0 per fit block, at least
constexpr int kFitBlocksMax = 512;      // fit blocks of one decomposition, at most (past 131 072 rows)
constexpr size_t kFitLdsMax = 64 * 1024;  // A^(1) staged in LDS by the fit kernel up to this

// Row stride (floats) of the transposed A^(1) the fit kernel stages in LDS:
// a multiple of 64 columns plus 4, so the 16 rank columns of a 128-bit read
// fall in distinct banks.
__host__ __device__ inline int fit_a0_stride(int I0) { return (I0 + 63) / 64 * 64 + 4; }

enum Op : int32_t { OP_STEP = 0, OP_SAMPLE = 1, OP_REPLAY = 2, OP_REFRESH = 3 };

// Device-resident state of one decomposition (first bytes of its workspace).
struct ChainState {
  int64_t t;          // steps taken
  int32_t status;     // sticky cpd_status of the device side
  int32_t done;       // batched/served members: stopped (target fit or step limit)
  double fit;         // last fit computed
  double x2;          // ||X||^2 of the stored tensor
  double inner;       // last <X, [[A]]>
  double xhat2;       // last ||[[A]]||^2
  int64_t ticks;      // wall-clock ticks of this chain's last step launch
  int64_t clock_start;  // wall clock when the distributions were first built
  int64_t clock_done;   // wall clock when done was set
  int64_t t_done;       // t when done was set
};

// Everything a kernel needs to run one decomposition.  Lives in device
// memory (inside the workspace); the batched and served paths keep arrays
// of these.
struct ChainDesc {
  int32_t N, R, B, RT;                 // RT = ceil(R / 16) MFMA row tiles
  int32_t dims[kMaxModes];
  int32_t ld[kMaxModes];               // row stride (elements) of copy n
  int32_t ksplit[kMaxModes];           // K-split of the contraction per mode
  int32_t vw[kMaxModes];               // output rows per lane in the contraction (1 or 2)
  int32_t dtype;                       // CPD_F32 or CPD_BF16 storage
  int32_t sampler, rule, nonneg;
  float alpha, eta, b;
  float pad1;
  double beta, gamma;
  uint64_t key0, key1;
  const void* X[kMaxModes];            // copy n: J_n rows x ld[n]
  float* A[kMaxModes];                 // factor k: dims[k] x R row-major
  float* S[kMaxModes];                 // AdaGrad accumulators, same shape
  double* C[kMaxModes];                // integer-valued CDF of mode k
  ChainState* state;
  double* parts;                       // kFitParts partial sums (fit / norm)
  int32_t active;                      // batched path: 0 = slot idle
  int32_t autostop;                    // fit kernels set state->done at the target
  int64_t step_limit;                  // stop stepping at this t (0 = none)
  double fit_target;                   // autostop: done once fit >= fit_target (if > 0)
};

struct StepArgs {
  int64_t nsteps;
  int32_t op;
  int32_t replay_mode;  // OP_REPLAY: the mode
  uint64_t sample_t;
  const int32_t* replay_idx;
  int32_t* out_idx;
  double* out_p;
  int32_t* out_mode;
  int32_t force_mode1;  // OP_STEP timing runs: 1 + the mode every step uses; 0 = drawn
  int32_t pad;
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11).  Step t, draw d uses counter
// (t, d / 4, 0, 0) under key (seed, stream_id) and output word d % 4.
// ---------------------------------------------------------------------------
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

__host__ __device__ inline uint64_t mulhi_u64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

__host__ __device__ inline void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1, uint64_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t lo0 = kPhiloxM0 * c0, hi0 = mulhi_u64(kPhiloxM0, c0);
    const uint64_t lo1 = kPhiloxM1 * c2, hi1 = mulhi_u64(kPhiloxM1, c2);
    const uint64_t y0 = hi1 ^ c1 ^ k0, y2 = hi0 ^ c3 ^ k1;
    c0 = y0;
    c1 = lo1;
    c2 = y2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

__host__ __device__ inline int bit_length_u32(uint32_t v) {
  int n = 0;
  while (v) {
    ++n;
    v >>= 1;
  }
  return n;
}

__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Pointers read from a descriptor are generic; accesses through them would
// be FLAT instructions, which also count against the LDS wait counter and so
// serialise LDS reads behind outstanding HBM loads.  gmem() marks them as
// global memory.
#define CPD_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ CPD_GLOBAL T* gmem(T* p) {
  return (CPD_GLOBAL T*)(p);
}
// The same for LDS pointers handed to a function that is not inlined (whose
// generic pointer parameters would otherwise become FLAT accesses).
#define CPD_LDS __attribute__((address_space(3)))
template <typename T>
__device__ __forceinline__ CPD_LDS T* lmem(T* p) {
  return (CPD_LDS T*)(p);
}

// Raises a kernel's dynamic-LDS limit once per device (bit d of *done set
// for device d; concurrent first calls may both set it, which is harmless).
inline hipError_t set_lds_limit_once(const void* fn, int bytes, std::atomic<uint32_t>* done) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const uint32_t bit = 1u << (dev & 31);
  if (done->load(std::memory_order_acquire) & bit) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) done->fetch_or(bit, std::memory_order_acq_rel);
  return e;
}

// Round an FP32 value to bfloat16, ties to even (NaN kept quiet).
__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

// Per-mode contraction split: the I_n x R output is cut into column tiles of
// 16 * VW entries (VW = 1 for FP32, 2 for BF16 storage), one tile per wave;
// with fewer tiles than waves the B dimension is split as well.
// Largest K-split of mode n's contraction the step kernel supports: every
// (row tile, K part) pair needs its own wave, and every part at least one
// chunk of fibres.
// Output rows per lane in the contraction of a mode of size In (a tile
// covers 16 * vw rows): BF16 reads element pairs, FP32 single elements
// (pairs of FP32 rows halve the tile count and unbalance the waves at the
// mode sizes of interest).
inline int host_vw(int In, int dtype) {
  (void)In;
  return dtype == CPD_BF16 ? 2 : 1;
}

// K-steps (four fibres each) per chunk of the contraction: the largest power
// of two within kChunkSteps / (VW * RT) register slots, so a chunk always
// divides the fibre padding kFibrePad.
__host__ __device__ constexpr int chunk_steps(int vw, int rt) {
  int u = kChunkSteps;
  while (u > 4 && u * vw * rt > kChunkSteps) u >>= 1;
  return u;
}

inline int max_ksplit(int In, int dtype, int B, int R) {
  const int vw = host_vw(In, dtype);
  const int nst = (In + 16 * vw - 1) / (16 * vw);
  const int rt = (R + 15) / 16;
  const int u = chunk_steps(vw, rt);
  const int chunks = (int)(((B + kFibrePad - 1) / kFibrePad) * kFibrePad / 4 / u);
  int m = kWaves / nst;
  if (m > chunks) m = chunks;
  return m < 1 ? 1 : m;
}

// Default K-split when no tuned value is given.
inline int host_ksplit(int In, int dtype, int B, int R) {
  const int vw = host_vw(In, dtype);
  const int nst = (In + 16 * vw - 1) / (16 * vw);
  if (nst >= kWaves) return 1;
  int ks = kWaves / nst;
  const int rt = (R + 15) / 16;
  const int u = chunk_steps(vw, rt);  // K-steps per chunk of the contraction
  const int chunks = (int)(((B + kFibrePad - 1) / kFibrePad) * kFibrePad / 4 / u);
  if (ks > chunks) ks = chunks;
  return ks < 1 ? 1 : ks;
}

// The Gram region of the leverage refresh: G (16 x 16), a pivot column and
// the pivots' reciprocals for one rank tile; R x R beyond.
__host__ __device__ constexpr int gram_doubles(int R, int RT) { return RT == 1 ? 288 : R * R; }

// The partials region of the persistent step: the Gs partials (256 floats
// per tile or wave) and the leverage refresh's Gram partials (doubles: one
// per thread, or kGramParts x 256 for one rank tile) share it.
__host__ __device__ constexpr size_t gram_part_bytes() {
  return sizeof(double) * (kBlock > 256 * kGramParts ? kBlock : 256 * kGramParts);
}
__host__ __device__ constexpr size_t chain_part_bytes(int RT) {
  const size_t gsp = sizeof(float) * 256 * (size_t)(RT * RT > kWaves ? RT * RT : kWaves);
  return gsp > gram_part_bytes() ? gsp : gram_part_bytes();
}

// LDS layout of the persistent step kernel for one descriptor, compiled for
// RT 16-row rank tiles (RT >= ceil(R / 16)).
struct LdsPlan {
  size_t cdf, idx, ratio, words, wf, rinv, rowoff, wht, gs, gsp, mbuf, gram, part, red, wts,
      misc, sbuf, fac, total;
  int rp16, bpad, ms, imax, sumdims, nd, nblk;
  int has_sbuf;  // AdaGrad accumulators of the updated mode staged in LDS
  int has_fac;   // every factor resident in LDS (sampled rows read from there)
};

__host__ __device__ inline LdsPlan lds_plan(int N, const int32_t* dims, int R, int B, int RT) {
  LdsPlan p;
  p.rp16 = 16 * RT;
  p.bpad = ((B + kFibrePad - 1) / kFibrePad) * kFibrePad;
  p.ms = p.rp16 + 1;
  p.imax = 0;
  p.sumdims = 0;
  for (int k = 0; k < N; ++k) {
    p.imax = dims[k] > p.imax ? dims[k] : p.imax;
    p.sumdims += dims[k];
  }
  p.nd = 1 + (N - 1) * B;
  p.nblk = (p.nd + 3) / 4;
  const int t2 = RT * RT;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (size_t)round_up((int64_t)bytes, 16);
    return o;
  };
  p.cdf = take(sizeof(double) * p.sumdims);
  p.idx = take(sizeof(int32_t) * (size_t)B * (N - 1));
  p.ratio = take(sizeof(double) * (size_t)B * (N - 1));
  p.words = take(sizeof(uint64_t) * 4 * (size_t)p.nblk);
  p.wf = take(sizeof(float) * p.bpad);
  p.rinv = take(sizeof(float) * p.bpad);
  p.rowoff = take(sizeof(uint32_t) * p.bpad);
  p.wht = take(sizeof(float) * (size_t)p.bpad * p.rp16);
  p.gs = take(sizeof(float) * (size_t)p.rp16 * p.rp16);
  p.mbuf = take(sizeof(float) * (size_t)p.imax * p.ms);
  p.gram = take(sizeof(double) * (size_t)gram_doubles(R, RT));
  // Gs partials (Gs phase) and the Gram partials (leverage refresh) share
  p.part = take(chain_part_bytes(RT));
  p.gsp = p.part;
  p.red = take(sizeof(double) * 2 * kWaves);
  p.wts = take(sizeof(double) * (size_t)p.imax);
  p.misc = take(sizeof(int32_t) * (8 + kMaxModes));
  // the AdaGrad accumulators of the mode being updated, when they fit
  const size_t sbytes = sizeof(float) * (size_t)p.imax * p.ms;
  p.has_sbuf = off + sbytes <= kLdsBudget;
  p.sbuf = p.has_sbuf ? take(sbytes) : 0;
  // all factors, compact rows (factor k at row offset sum_{m<k} dims[m])
  const size_t fbytes = sizeof(float) * (size_t)p.sumdims * R;
  p.has_fac = off + fbytes <= kLdsBudget;
  p.fac = p.has_fac ? take(fbytes) : 0;
  p.total = off;
  return p;
}

}  // namespace cpdmi
