// Host and device definitions of the grid-wide step (large mini-batches):
// slice sizes, the fibre-range split of a gather block, the hand-over
// between its three kernels and their LDS maps.
#pragma once

#include "cpd_internal.hpp"

namespace cpdmi {

// ---------------------------------------------------------------------------
// Grid-wide step (large mini-batches): every block of the gather kernel
// takes a slice of up to kWideFibresMax sampled fibres.
// ---------------------------------------------------------------------------
constexpr int kWideFibresMax = 512;
constexpr int kGatherThreads = 512;  // threads of a gather block
constexpr int kGatherWaves = kGatherThreads / 64;
constexpr int kGatherBufs = 2;  // register buffers of fibre chunks per wave
// Gs rows are 16 RT + kGsPad floats apart in the gather kernel's LDS (rows
// 16 RT floats apart put the 16 rows an epilogue read spans in one bank).
constexpr int kGsPad = 4;

// Fibres per block of the gather kernel for mini-batch B: about 256 blocks
// while the slices stay within [128, 512] fibres (measured on 300-element
// fibres: fewer, longer slices win up to 512 fibres, more blocks beyond).
inline int wide_fibres(int B) {
  int fb = (int)round_up((B + 255) / 256, kFibrePad);
  if (fb < kFibrePad) fb = kFibrePad;
  if (fb > kWideFibresMax) fb = kWideFibresMax;
  return fb;
}

// Fibre-range split of a gather block's contraction for a mode of nst
// output tiles: with fewer tiles than waves, the 8 waves form 8 / kp tile
// groups times kp parts of the slice's nck chunks (so every wave has work);
// kp = 1 otherwise (one wave per tile over all the fibres measured faster
// than any split once every wave has a tile).  Each (block, part) writes its
// own part of -G^T.
constexpr int kWideMaxParts = 8;
__host__ __device__ inline int wide_kparts(int nst, int nck) {
  int kp = 1;
  while (kp < kWideMaxParts && nst * kp * 2 <= kGatherWaves && kp * 2 <= nck) kp *= 2;
  return kp;
}

// Gather blocks per slice.  With fewer slices than CUs the row tiles of
// the updated mode are dealt over several blocks of the same slice (each
// repeats the slice's draws, WH rows and Gs), up to one block per CU in all,
// so that a small mini-batch is not a few CUs' work; a tile's arithmetic is
// the same whichever block runs it, and the blocks of a slice write
// disjoint rows of the slice's parts.  (Measured on the 300^3 step: 64
// blocks in all left B = 8192 at 18.5 us, 256 give 15.7 us, 512 give 20.2.)
constexpr int kWideTileSplitMax = 16;
constexpr int kWideSplitBlocks = 256;
inline int wide_tsplit(int nslices) {
  int g = 1;
  while (g < kWideTileSplitMax && nslices * g * 2 <= kWideSplitBlocks) g *= 2;
  return g;
}

// Mode and step of the step in flight, written by the gather kernel for the
// update and refresh kernels that follow it on the stream.
struct WideInfo {
  int64_t t;
  int32_t n;
  int32_t pad;
};

struct WideArgs {
  int32_t op;           // OP_STEP, OP_SAMPLE or OP_REPLAY
  int32_t replay_mode;  // OP_REPLAY: the mode
  int32_t force_mode1;  // OP_STEP timing runs: 1 + the mode every step uses; 0 = drawn
  int32_t fb;           // fibres per slice (a multiple of kFibrePad)
  int32_t tsplit;       // gather blocks per slice (wide_tsplit)
  uint64_t sample_t;
  const int32_t* replay_idx;
  int32_t* out_idx;
  double* out_p;
  int32_t* out_mode;
  float* part;          // per block: -G^T, R x I_n (row r holds the I_n entries)
  WideInfo* info;
};

// LDS map of the gather kernel (one slice of fb fibres).
struct GatherPlan {
  size_t cdf, idx, ratio, words, wf, rinv, rowoff, wht, gs, gsp, misc, total;
  int nwb;  // Philox blocks per mode slot
};

__host__ __device__ inline GatherPlan gather_plan(int N, const int32_t* dims, int RT, int fb) {
  GatherPlan p;
  int sumdims = 0;
  for (int k = 0; k < N; ++k) sumdims += dims[k];
  const int nm1 = N - 1, rp16 = 16 * RT, t2 = RT * RT;
  p.nwb = fb / 4 + 2;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (size_t)round_up((int64_t)bytes, 16);
    return o;
  };
  p.cdf = take(sizeof(double) * sumdims);
  p.idx = take(sizeof(int32_t) * (size_t)fb * nm1);
  p.ratio = take(sizeof(double) * (size_t)fb * nm1);
  p.words = take(sizeof(uint64_t) * 4 * (size_t)p.nwb * nm1);
  p.wf = take(sizeof(float) * fb);
  p.rinv = take(sizeof(float) * fb);
  p.rowoff = take(sizeof(uint32_t) * fb);
  p.wht = take(sizeof(float) * (size_t)fb * rp16);
  p.gs = take(sizeof(float) * (size_t)rp16 * (rp16 + kGsPad));
  // Gs partials only when fewer tiles than waves split the fibres (with at
  // least as many tiles as waves every tile is written straight to gs)
  p.gsp = take(t2 >= kGatherWaves ? 0 : sizeof(float) * 256 * (size_t)kGatherWaves);
  p.misc = take(sizeof(int32_t) * (8 + kMaxModes));
  p.total = off;
  return p;
}

// LDS map of the refresh kernel (the CDF of one mode at a time).  The Gram
// of the leverage scores is planned for R <= 64 (the sampler is refused
// beyond).  The factor rows are staged in LDS (mbuf) for R <= 64, and
// beyond when they fit; otherwise (rows_in_lds = 0) the row sums are read
// straight from global memory.
struct RefreshPlan {
  size_t cdf, mbuf, gram, part, red, wts, misc, total;
  int ms, imax, rows_in_lds;
};

__host__ __device__ inline RefreshPlan refresh_plan(int N, const int32_t* dims, int R, int RT) {
  RefreshPlan p;
  p.imax = 0;
  for (int k = 0; k < N; ++k) p.imax = dims[k] > p.imax ? dims[k] : p.imax;
  p.ms = 16 * RT + 1;
  const bool small_rank = R <= 16 * kMaxRankTiles;
  for (int pass = 0; pass < 2; ++pass) {
    p.rows_in_lds = pass == 0;
    size_t off = 0;
    auto take = [&](size_t bytes) {
      size_t o = off;
      off += (size_t)round_up((int64_t)bytes, 16);
      return o;
    };
    p.cdf = take(sizeof(double) * p.imax);
    p.mbuf = take(p.rows_in_lds ? sizeof(float) * (size_t)p.imax * p.ms : 0);
    p.gram = take(small_rank ? sizeof(double) * (size_t)gram_doubles(R, RT) : 0);
    p.part = take(gram_part_bytes());
    p.red = take(sizeof(double) * 2 * kWaves);
    p.wts = take(sizeof(double) * (size_t)p.imax);
    p.misc = take(sizeof(int32_t) * (8 + kMaxModes));
    p.total = off;
    if (small_rank || off <= kLdsBudget) break;
  }
  return p;
}

}  // namespace cpdmi
