// Persistent step kernel: one 512-thread workgroup advances one
// decomposition by many SGD steps without leaving the chip.
//
// One step (paper Section 3, Algorithms 3-5):
//   1. mode draw and inverse-CDF sampling of B rows of every mode k != n
//      from the integer-valued CDFs held in LDS (Philox4x64-10 words,
//      Lemmas 2 and 4); one thread per draw.  The Philox words of the next
//      step are generated ahead by threads that are idle in phase 2.
//   2. one thread per sampled fibre: p_f = prod_k q_k(i_k)/Q_k,
//      w_f = 1/(B p_f), the fibre's row in copy n (unfolding index map) and
//      the sampled KRP row H(f,:) = Hadamard product of factor rows, written
//      as WH in the A-operand layout of the matrix-core instruction.
//   3. Gs = (WH)^T H on the matrix cores, the fibre dimension split over
//      the waves and the partial tiles summed in a fixed order.
//   4. on the matrix cores (v_mfma_f32_16x16x4f32; BF16 storage with up to
//      two rank tiles: v_mfma_f32_16x16x32_bf16 with WH as three BF16 terms),
//      per 16-column tile of the I_n x R output:
//      -G^T = (WH)^T X_s - Gs^T A^(n)T, the fibres streamed
//      from HBM straight into the B operand with two register buffers; the
//      tile's lanes then apply the fixed, decreasing or AdaGrad update
//      (optional projection onto A >= 0) to the entries they hold.
//   5. the CDF of mode n from the new factor: squared row norms, or leverage
//      scores from an FP64 Gram, a one-wave Cholesky and a forward solve per
//      row; quantised to exact integers and prefix-summed.
#include "step_common.hpp"

namespace cpdmi {

// A^(n) into mbuf (row i at mbuf[i * ms]) for the contraction epilogue, in
// two halves so the loads can be in flight while the draws are searched:
// prefetch_issue loads the first kPrefetch * kBlock entries into registers,
// prefetch_commit stores them (and any further rows).  The rank padding
// columns of mbuf are zeroed once per launch: nothing writes them.
constexpr int kPrefetch = 4;
__device__ __forceinline__ void prefetch_issue(const ChainDesc* dp, const Smem& S, int n,
                                               float (&v)[kPrefetch], float (&sv)[kPrefetch]) {
  const int total = dp->dims[n] * dp->R;
  const CPD_GLOBAL float* An = gmem(dp->A[n]);
  const CPD_GLOBAL float* Sn = gmem(dp->S[n]);
  const bool ss = S.has_sbuf && dp->rule == CPD_RULE_ADAGRAD;
  const float* Af = S.fac() + S.coff()[n] * dp->R;
#pragma unroll
  for (int j = 0; j < kPrefetch; ++j) {
    const int e = threadIdx.x + j * kBlock;
    v[j] = e < total ? (S.has_fac ? Af[e] : An[e]) : 0.f;
    sv[j] = (ss && e < total) ? Sn[e] : 0.f;
  }
}

__device__ __forceinline__ void prefetch_commit(const ChainDesc* dp, const Smem& S, int n,
                                                const float (&v)[kPrefetch],
                                                const float (&sv)[kPrefetch]) {
  const int R = dp->R, In = dp->dims[n], total = In * R, ms = S.ms;
  float* mbuf = S.mbuf();
  float* sbuf = S.sbuf();
  const bool ss = S.has_sbuf && dp->rule == CPD_RULE_ADAGRAD;
#pragma unroll
  for (int j = 0; j < kPrefetch; ++j) {
    const int e = threadIdx.x + j * kBlock;
    if (e < total) {
      const int i = e / R;
      mbuf[i * ms + (e - i * R)] = v[j];
      if (ss) sbuf[i * ms + (e - i * R)] = sv[j];
    }
  }
  const CPD_GLOBAL float* An = gmem(dp->A[n]);
  const CPD_GLOBAL float* Sn = gmem(dp->S[n]);
  const float* Af = S.fac() + S.coff()[n] * R;
  // the rest in rounds whose loads are all issued before the first store
  for (int e0 = threadIdx.x + kPrefetch * kBlock; e0 < total; e0 += kPrefetch * kBlock) {
    float a[kPrefetch], b[kPrefetch];
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) {
      const int e = e0 + j * kBlock;
      a[j] = e < total ? (S.has_fac ? Af[e] : An[e]) : 0.f;
      b[j] = (ss && e < total) ? Sn[e] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) {
      const int e = e0 + j * kBlock;
      if (e < total) {
        const int i = e / R;
        mbuf[i * ms + (e - i * R)] = a[j];
        if (ss) sbuf[i * ms + (e - i * R)] = b[j];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Contraction and update for mode n.  Per 16-column tile (columns col0 +
// j*VW + v of the I_n x R output), K = padded fibres:
//   A operand: lane l holds WH[f0 + l/16][rt*16 + l%16]   (LDS)
//   B operand: lane l holds X_s[f0 + l/16][col0 + (l%16)*VW + v]   (HBM)
// followed by K = rank (steps of 4) with A = -Gs[rt*16 + l%16][s0 + l/16]
// and B = A^(n)[col0 + (l%16)*VW + v][s0 + l/16], which leaves -G^T in the
// accumulators.  A wave walks all K-chunks of all its tiles as one stream
// with two register buffers.
// ---------------------------------------------------------------------------
template <int VW, int RT, bool BF16>
__device__ __forceinline__ bool contract_update(const ChainDesc* dp, const Smem& S, int n, uint64_t t) {
  constexpr int U = chunk_steps(VW, RT);  // K-steps per part of the fibre range
  const int lane = threadIdx.x & 63;
  const int wave = uniform_int(threadIdx.x >> 6);
  const int fl = lane >> 4, cl = lane & 15;
  const int In = dp->dims[n], R = dp->R, ms = S.ms, rp16 = S.rp16;
  const int SW = 16 * VW;
  const int nst = (In + SW - 1) / SW;
  const int ks = dp->ksplit[n];
  const int nck_all = S.bpad / (4 * U);  // bpad is a multiple of 4 * kChunkSteps
  const float* __restrict__ wht = S.wht();
  const uint32_t* __restrict__ rowb = S.rowb();
  const CPD_GLOBAL char* __restrict__ Xb = gmem((const char*)dp->X[n]);
  CPD_GLOBAL float* An = gmem(dp->A[n]);
  CPD_GLOBAL float* Sn = gmem(dp->S[n]);
  const bool ada = dp->rule == CPD_RULE_ADAGRAD;
  const UpdateParams up = update_params(dp, t);
  float* mbuf = S.mbuf();

  int nitems, c0, c1, st_first, kc = 0;
  if (ks <= 1) {
    nitems = wave < nst ? (nst - 1 - wave) / kWaves + 1 : 0;
    c0 = 0;
    c1 = nck_all;
    st_first = wave;
  } else {
    kc = wave / nst;
    nitems = wave < nst * ks ? 1 : 0;
    c0 = kc * nck_all / ks;
    c1 = (kc + 1) * nck_all / ks;
    st_first = wave % nst;
  }
  const int nck = c1 - c0;
  // the tile's lanes update their entries directly when the whole fibre
  // range is theirs and the AdaGrad accumulators are staged in LDS;
  // otherwise -G^T goes to mbuf and an element-wise pass updates
  const bool direct = ks <= 1 && S.has_sbuf;
  bool bad = false;

  f4 acc[RT][VW];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int v = 0; v < VW; ++v) acc[rt][v] = f4{0.f, 0.f, 0.f, 0.f};
  // -Gs^T A^T added to the accumulators of tile st
  auto add_ags = [&](int st) {
    const int col0 = st * SW;
#pragma unroll
    for (int kk = 0; kk < 4 * RT; ++kk) {
      const int s = 4 * kk + fl;
      float bA[VW];
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        // rows past I_n only feed output columns that are never stored;
        // rank columns past R are zero in the prefetched rows
        const int i = col0 + cl * VW + v;
        bA[v] = mbuf[(i < In ? i : In - 1) * ms + s];
      }
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const float a = -S.gs()[(rt * 16 + cl) * rp16 + s];
#pragma unroll
        for (int v = 0; v < VW; ++v)
          acc[rt][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bA[v], acc[rt][v], 0, 0, 0);
      }
    }
  };
  // -G^T of tile st into mbuf (the tile's rows were only read by this wave)
  auto store_neg_g = [&](int st) {
    const int col0 = st * SW;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < VW; ++v)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = rt * 16 + 4 * fl + q;
          const int i = col0 + cl * VW + v;
          if (r < R && i < In) mbuf[i * ms + r] = acc[rt][v][q];
        }
  };
  // the update of the entries of tile st that this lane holds
  auto update_tile = [&](int st) {
    const int col0 = st * SW;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < VW; ++v)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = rt * 16 + 4 * fl + q;
          const int i = col0 + cl * VW + v;
          if (r < R && i < In) {
            // LDS only: a global store here would queue behind the fibre
            // loads in flight; the rows are written back after the phase
            const float g = -acc[rt][v][q];
            float sacc = ada ? S.sbuf()[i * ms + r] : 0.f;
            const float an = update_entry(up, mbuf[i * ms + r], g, sacc);
            if (ada) S.sbuf()[i * ms + r] = sacc;
            if (!isfinite(an)) bad = true;
            mbuf[i * ms + r] = an;
          }
        }
  };
  // The wave's work is a stream of chunks (U K-steps each) over its items;
  // two register buffers: the loads of chunk c+1 are in flight while chunk
  // c is multiplied.  Two accumulator sets (even / odd K-steps) halve the
  // dependent-accumulation chain.
  f4 acc2[RT][VW];
  float xbuf[kFibreBufs][U][VW];
  auto load = [&](float (&x)[U][VW], int c) {
    const int it = c / nck;
    const int st = st_first + it * kWaves;
    const int kq0 = (c0 + (c - it * nck)) * (U / 4);  // first group of 4 K-steps
    const uint32_t colb = (uint32_t)((st * SW + cl * VW) * (BF16 ? 2 : 4));
#pragma unroll
    for (int u4 = 0; u4 < U / 4; ++u4) {
      const uint4 ob = *(const uint4*)(rowb + (kq0 + u4) * 16 + fl * 4);
      const uint32_t o4[4] = {ob.x, ob.y, ob.z, ob.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const CPD_GLOBAL char* p = Xb + (o4[j] + colb);
        const int u = 4 * u4 + j;
        if constexpr (BF16) {
          if constexpr (VW == 2) {
            const uint32_t pk = *(const CPD_GLOBAL uint32_t*)p;
            x[u][0] = __uint_as_float(pk << 16);
            x[u][1] = __uint_as_float(pk & 0xFFFF0000u);
          } else {
            x[u][0] = bf16_to_f32(*(const CPD_GLOBAL uint16_t*)p);
          }
        } else {
          if constexpr (VW == 2) {
            const uint64_t v2 = *(const CPD_GLOBAL uint64_t*)p;
            x[u][0] = __uint_as_float((uint32_t)v2);
            x[u][1] = __uint_as_float((uint32_t)(v2 >> 32));
          } else {
            x[u][0] = *(const CPD_GLOBAL float*)p;
          }
        }
      }
    }
  };
  auto compute = [&](const float (&x)[U][VW], int c) {
    const int it = c / nck;
    const int ci = c - it * nck;
    const int st = st_first + it * kWaves;
    const int kq0 = (c0 + ci) * (U / 4);
    if (ci == 0) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int v = 0; v < VW; ++v) {
          acc[rt][v] = f4{0.f, 0.f, 0.f, 0.f};
          acc2[rt][v] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    // all A operands of the chunk first: one wait for the LDS reads, not one
    // per group of four K-steps
    f4 wa[U / 4][RT];
#pragma unroll
    for (int u4 = 0; u4 < U / 4; ++u4)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        wa[u4][rt] = *(const f4*)(wht + ((kq0 + u4) * RT + rt) * 256 + lane * 4);
    if constexpr (BF16 && U % 8 == 0) {
      mfma_wh_x_bf16<U, RT, VW>(wa, x, acc, acc2);
    } else {
#pragma unroll
      for (int u4 = 0; u4 < U / 4; ++u4) {
        const f4* a4 = wa[u4];
#pragma unroll
        for (int j = 0; j < 4; j += 2)
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int v = 0; v < VW; ++v) {
              acc[rt][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[rt][j], x[4 * u4 + j][v],
                                                                acc[rt][v], 0, 0, 0);
              acc2[rt][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                  a4[rt][j + 1], x[4 * u4 + j + 1][v], acc2[rt][v], 0, 0, 0);
            }
      }
    }
    if (ci == nck - 1) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[rt][v] += acc2[rt][v];
      if (ks <= 1) {
        add_ags(st);
        if (direct) update_tile(st);
        else store_neg_g(st);
      }
    }
  };
  const int total = nitems * nck;
  if (total > 0) {
    // kFibreBufs register buffers: the loads of the next kFibreBufs - 1
    // chunks are in flight while a chunk is multiplied
#pragma unroll
    for (int j = 0; j < kFibreBufs - 1; ++j)
      if (j < total) load(xbuf[j], j);
    // The loads are issued unconditionally (past the end they repeat the
    // last chunk and are never used), so the loop body is straight-line and
    // the compiler's waits on the load counter stay one chunk behind
    // (measured: 0.6 us of 19 per step at 300^3).
    int c = 0;
    for (; c + kFibreBufs - 1 < total; c += kFibreBufs) {
#pragma unroll
      for (int j = 0; j < kFibreBufs; ++j) {
        const int nx = c + j + kFibreBufs - 1;
        load(xbuf[(j + kFibreBufs - 1) % kFibreBufs], nx < total ? nx : total - 1);
        compute(xbuf[j], c + j);
      }
    }
#pragma unroll
    for (int j = 0; j < kFibreBufs - 1; ++j)
      if (c + j < total) compute(xbuf[j], c + j);
  }
  if (ks > 1) {
    // K-split: the first part adds -Gs^T A^T, the partial tiles are summed
    // in a fixed order (one part per round)
    if (nitems && kc == 0) add_ags(st_first);
    __syncthreads();  // every add_ags read of the prefetched rows is done
    for (int round = 0; round < ks; ++round) {
      if (nitems && kc == round) {
        const int col0 = st_first * SW;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int v = 0; v < VW; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int r = rt * 16 + 4 * fl + q;
              const int i = col0 + cl * VW + v;
              if (r < R && i < In) {
                float* m = mbuf + i * ms + r;
                *m = round ? *m + acc[rt][v][q] : acc[rt][v][q];
              }
            }
      }
      __syncthreads();
    }
  } else if (!direct) {
    __syncthreads();
  }
  if (direct) {
    // write the updated rows (and accumulators) back, coalesced
    __syncthreads();
    float* Af = S.fac() + S.coff()[n] * R;
    for (int e = threadIdx.x; e < In * R; e += kBlock) {
      const int i = e / R, r = e - i * R;
      const float a = mbuf[i * ms + r];
      An[e] = a;
      if (S.has_fac) Af[e] = a;
      if (ada) Sn[e] = S.sbuf()[i * ms + r];
    }
  } else {
    // element-wise update from -G^T in mbuf
    float* Af = S.fac() + S.coff()[n] * R;
    for (int e = threadIdx.x; e < In * R; e += kBlock) {
      const int i = e / R, r = e - i * R;
      const float g = -mbuf[i * ms + r];
      float sacc = ada ? Sn[e] : 0.f;
      const float an = update_entry(up, S.has_fac ? Af[e] : An[e], g, sacc);
      if (ada) Sn[e] = sacc;
      if (!isfinite(an)) bad = true;
      An[e] = an;
      if (S.has_fac) Af[e] = an;
      mbuf[i * ms + r] = an;
    }
  }
  return bad;
}

// The BF16 contraction as a call of its own: it then gets the whole
// register file instead of sharing it with the rest of the step, which
// schedules it better (measured).
template <int RT>
__device__ __noinline__ bool contract_update_bf16(const ChainDesc* dp, const Smem& S, int n,
                                                  uint64_t t) {
  return contract_update<2, RT, true>(dp, S, n, t);
}

// WH rows of the sampled fibres, CPI columns per item (one rank tile holds
// 16 / CPI items).  Factor rows come from the resident LDS copy when there
// is one.
template <int CPI, int RT>
__device__ __forceinline__ void krp_rows(const ChainDesc* dp, const Smem& S, int n, int B, int nm1,
                                         float* wht) {
  const int R = dp->R;
  constexpr int ipf = 16 * RT / CPI;
  for (int itm = threadIdx.x; itm < S.bpad * ipf; itm += kBlock) {
    const int f = itm / ipf, c0 = (itm - f * ipf) * CPI;
    float h[CPI];
#pragma unroll
    for (int c = 0; c < CPI; ++c) h[c] = 0.f;
    float wfl = 0.f;
    if (f < B) {
      double p = 1.0;
      for (int sl = 0; sl < nm1; ++sl) p = p * S.ratio()[sl * B + f];
      wfl = (float)(1.0 / ((double)B * p));
      for (int q = 0; q < nm1; ++q) {
        const int k = q < n ? q : q + 1;
        const int i = S.idx()[f * nm1 + q];
        float v[CPI];
        if (S.has_fac) {
          const float* row = S.fac() + (S.coff()[k] + i) * R;
#pragma unroll
          for (int c = 0; c < CPI; ++c) v[c] = c0 + c < R ? row[c0 + c] : 0.f;
        } else {
          const CPD_GLOBAL float* row = gmem(dp->A[k]) + (int64_t)i * R;
#pragma unroll
          for (int c = 0; c < CPI; ++c) v[c] = c0 + c < R ? row[c0 + c] : 0.f;
        }
#pragma unroll
        for (int c = 0; c < CPI; ++c) h[c] = q == 0 ? v[c] : h[c] * v[c];
      }
    }
    const int k4 = f >> 2, g4 = f & 3;
#pragma unroll
    for (int c = 0; c < CPI; ++c) {
      const int col = c0 + c;
      wht[wht_index(k4, col >> 4, g4 * 16 + (col & 15), RT)] = wfl * h[c];
    }
  }
}

// RT: number of 16-row rank tiles the kernel is compiled for; a chain with
// fewer tiles runs with zero-padded rank columns.
template <int RT>
__global__ void __launch_bounds__(kBlock) chain_kernel(const ChainDesc* __restrict__ descs,
                                                       StepArgs args) {
  const ChainDesc* dp = descs + blockIdx.x;
  if (!dp->active) return;
  ChainState* st = dp->state;
  if (args.op != OP_SAMPLE && args.op != OP_REFRESH && st->status != 0) return;
  if (args.op == OP_STEP && (st->done || args.force_mode1 > dp->N)) return;
  const int64_t clock0 = (int64_t)wall_clock64();
  const int tid = threadIdx.x;
  const int N = dp->N, R = dp->R, B = dp->B;
  const LdsPlan P = lds_plan(N, dp->dims, R, B, RT);
  Smem S;
  S.o_cdf = P.cdf;
  S.o_idx = P.idx;
  S.o_ratio = P.ratio;
  S.o_words = P.words;
  S.o_wf = P.wf;
  S.o_rinv = P.rinv;
  S.o_rowoff = P.rowoff;
  S.o_wht = P.wht;
  S.o_gs = P.gs;
  S.o_gsp = P.gsp;
  S.o_mbuf = P.mbuf;
  S.o_gram = P.gram;
  S.o_part = P.part;
  S.o_red = P.red;
  S.o_wts = P.wts;
  S.o_misc = P.misc;
  S.o_sbuf = P.sbuf;
  S.has_sbuf = P.has_sbuf;
  S.o_fac = P.fac;
  S.has_fac = P.has_fac;
  S.rp16 = P.rp16;
  S.bpad = P.bpad;
  S.ms = P.ms;
  S.nd = P.nd;
  S.nblk = P.nblk;
  if (tid < 8) S.misc()[tid] = 0;
  // rank padding columns of the staged factor rows: read by the matrix-core
  // epilogue as zeros, never written by a step
  {
    const int padc = P.ms - R;
    for (int e = tid; e < P.imax * padc; e += kBlock) {
      const int i = e / padc;
      ((float*)(cpd_smem + P.mbuf))[i * P.ms + R + (e - i * padc)] = 0.f;
    }
  }
  if (tid == 0) {
    int o = 0;
    for (int k = 0; k < N; ++k) {
      S.coff()[k] = o;
      o += dp->dims[k];
    }
  }
  __syncthreads();
  for (int k = 0; k < N; ++k)
    for (int i = tid; i < dp->dims[k]; i += kBlock) S.cdf()[S.coff()[k] + i] = gmem(dp->C[k])[i];
  if (S.has_fac && args.op != OP_REFRESH)
    for (int k = 0; k < N; ++k) {
      const CPD_GLOBAL float* Ak = gmem(dp->A[k]);
      float* dst = S.fac() + S.coff()[k] * R;
      for (int e = tid; e < dp->dims[k] * R; e += kBlock) dst[e] = Ak[e];
    }

  if (args.op == OP_REFRESH) {
    __syncthreads();
    int err = 0;
    for (int n = 0; n < N && !err; ++n) {
      for (int e = tid; e < dp->dims[n] * R; e += kBlock) {
        const int i = e / R, r = e - i * R;
        S.mbuf()[i * S.ms + r] = gmem(dp->A[n])[e];
      }
      __syncthreads();
      err = refresh_cdf<RT>(dp, S, n, S.mbuf(), S.ms);
      __syncthreads();
    }
    if (tid == 0) {
      if (err) st->status = err;
      if (st->clock_start == 0) st->clock_start = clock0;
    }
    return;
  }

  const int64_t t0 = args.op == OP_SAMPLE ? (int64_t)args.sample_t : st->t;
  int64_t nsteps = args.op == OP_STEP ? args.nsteps : 1;
  if (args.op == OP_STEP && dp->step_limit > 0 && t0 + nsteps > dp->step_limit)
    nsteps = dp->step_limit > t0 ? dp->step_limit - t0 : 0;
  const int nm1 = N - 1;
  const int nd = S.nd, nblk = S.nblk;
  // threads with no fibre in phase 2 generate the next step's Philox blocks
  const int npre_max = kBlock > S.bpad ? (kBlock - S.bpad < nblk ? kBlock - S.bpad : nblk) : 0;
  uint64_t* words = S.words();
  int64_t done = 0;
  int err = 0;

  for (int64_t s = 0; s < nsteps; ++s) {
    const uint64_t t = (uint64_t)(t0 + s);
    // ---- 1. draws ------------------------------------------------------
    int n;
    if (args.op == OP_REPLAY) {
      n = args.replay_mode;
      float pv[kPrefetch], ps[kPrefetch];
      prefetch_issue(dp, S, n, pv, ps);
      prefetch_commit(dp, S, n, pv, ps);
      // caller-supplied indices: reject any outside its mode's range
      for (int e = tid; e < B * nm1; e += kBlock) {
        const int f = e / nm1, sl = e - f * nm1;
        const int k = sl < n ? sl : sl + 1;
        int i = gmem(args.replay_idx)[e];
        if (i < 0 || i >= dp->dims[k]) {
          S.misc()[1] = CPD_E_INVALID;
          i = 0;
        }
        S.idx()[e] = i;
        const double* Ck = S.cdf() + S.coff()[k];
        const double Q = Ck[dp->dims[k] - 1];
        S.ratio()[sl * B + f] = (Ck[i] - (i ? Ck[i - 1] : 0.0)) / Q;
      }
    } else {
      const int npre = S.misc()[4];
      if (npre < nblk) {
        for (int b = npre + tid; b < nblk; b += kBlock) {
          uint64_t o[4];
          philox4x64_10(t, (uint64_t)b, 0, 0, dp->key0, dp->key1, o);
          words[4 * b + 0] = o[0];
          words[4 * b + 1] = o[1];
          words[4 * b + 2] = o[2];
          words[4 * b + 3] = o[3];
        }
        __syncthreads();
      }
      n = args.force_mode1 ? args.force_mode1 - 1 : (int)mulhi_u64(words[0], (uint64_t)N);
      float pv[kPrefetch], ps[kPrefetch];
      prefetch_issue(dp, S, n, pv, ps);
      for (int d = 1 + tid; d < nd; d += kBlock) {
        const int sl = (d - 1) / B, f = (d - 1) - sl * B;
        const int k = sl < n ? sl : sl + 1;
        const double* Ck = S.cdf() + S.coff()[k];
        const int Ik = dp->dims[k];
        const double Q = Ck[Ik - 1];
        const int i = cdf_search(Ck, Ik, (double)mulhi_u64(words[d], (uint64_t)Q));
        S.idx()[f * nm1 + sl] = i;
        S.ratio()[sl * B + f] = (Ck[i] - (i ? Ck[i - 1] : 0.0)) / Q;
      }
      prefetch_commit(dp, S, n, pv, ps);
    }
    __syncthreads();
    if (S.misc()[1]) {
      err = S.misc()[1];
      break;
    }
    if (tid == 0) S.misc()[4] = 0;
    // ---- 2. per fibre: p_f, w_f, row offset; WH rows 4 columns per item ----
    const int ldn = dp->ld[n];
    const int64_t esz = dp->dtype == CPD_BF16 ? 2 : 4;
    float* wht = S.wht();
    for (int f = tid; f < S.bpad; f += kBlock) {
      const int ro = (f >> 4) * 16 + (f & 3) * 4 + ((f >> 2) & 3);
      if (f < B) {
        double p = 1.0;
        int64_t j = 0, stride = 1;
        int sl = 0;
        for (int k = 0; k < N; ++k) {
          if (k == n) continue;
          p = p * S.ratio()[sl * B + f];
          j += (int64_t)S.idx()[f * nm1 + sl] * stride;
          stride *= dp->dims[k];
          ++sl;
        }
        S.wf()[f] = (float)(1.0 / ((double)B * p));
        S.rinv()[f] = (float)((double)B * p);
        S.rowb()[ro] = (uint32_t)(j * ldn * esz);
        if (args.op == OP_SAMPLE) {
          gmem(args.out_p)[f] = p;
          for (int q = 0; q < nm1; ++q) gmem(args.out_idx)[f * nm1 + q] = S.idx()[f * nm1 + q];
        }
      } else {
        S.wf()[f] = 0.f;
        S.rinv()[f] = 0.f;
        S.rowb()[ro] = 0;
      }
    }
    // sampled KRP row H(f, c) = prod over k != n (ascending) of A^(k)(i_k, c),
    // scaled by w_f (recomputed here exactly as above); items of 4, 8 or 16
    // columns so that about one item per thread covers the batch
    {
      const int work = S.bpad * RT;
      if (work >= kBlock) krp_rows<16, RT>(dp, S, n, B, nm1, wht);
      else if (work >= kBlock / 2) krp_rows<8, RT>(dp, S, n, B, nm1, wht);
      else krp_rows<4, RT>(dp, S, n, B, nm1, wht);
    }
    if (args.op == OP_SAMPLE) {
      if (tid == 0) *gmem(args.out_mode) = n;
      return;
    }
    if (args.op == OP_STEP && npre_max > 0 && s + 1 < nsteps && tid >= S.bpad &&
        tid - S.bpad < npre_max) {
      // this step's words are consumed; generate the next step's
      const int b = tid - S.bpad;
      uint64_t o[4];
      philox4x64_10(t + 1, (uint64_t)b, 0, 0, dp->key0, dp->key1, o);
      words[4 * b + 0] = o[0];
      words[4 * b + 1] = o[1];
      words[4 * b + 2] = o[2];
      words[4 * b + 3] = o[3];
      if (b == 0) S.misc()[4] = npre_max;
    }
    __syncthreads();
    // ---- 3. Gs ----------------------------------------------------------
    compute_gs<RT>(S);
    // ---- 4. contraction and update -----------------------------------------
    bool bad;
    if (dp->dtype == CPD_BF16) bad = contract_update_bf16<RT>(dp, S, n, t);
    else bad = contract_update<1, RT, false>(dp, S, n, t);
    if (bad) S.misc()[1] = CPD_E_DIVERGED;
    __syncthreads();
    ++done;
    if (S.misc()[1]) {
      err = S.misc()[1];
      break;
    }
    // ---- 5. distribution of mode n from the new factor -------------------
    if (dp->sampler != CPD_SAMPLER_UNIFORM) {
      err = refresh_cdf<RT>(dp, S, n, S.mbuf(), S.ms);
      if (err) break;
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (args.op == OP_STEP || args.op == OP_REPLAY) st->t = t0 + done;
    if (err) st->status = err;
    if (args.op == OP_STEP) st->ticks = (int64_t)wall_clock64() - clock0;
  }
}

// Host-side launcher (declared in cpd_runtime.hpp).  rt = the largest
// number of rank tiles among the descriptors.
template <int RT>
static hipError_t launch_rt(const ChainDesc* descs, int nchains, size_t lds_bytes,
                            const StepArgs& args, hipStream_t stream) {
  static std::atomic<uint32_t> attr_set{0};
  hipError_t e = set_lds_limit_once((const void*)chain_kernel<RT>, 160 * 1024, &attr_set);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(chain_kernel<RT>, dim3(nchains), dim3(kBlock), lds_bytes, stream, descs, args);
  return hipGetLastError();
}

hipError_t launch_chain_kernel(const ChainDesc* descs, int nchains, int rt, size_t lds_bytes,
                               const StepArgs& args, hipStream_t stream) {
  switch (rt) {
    case 1: return launch_rt<1>(descs, nchains, lds_bytes, args, stream);
    case 2: return launch_rt<2>(descs, nchains, lds_bytes, args, stream);
    case 3: return launch_rt<3>(descs, nchains, lds_bytes, args, stream);
    default: return launch_rt<4>(descs, nchains, lds_bytes, args, stream);
  }
}

}  // namespace cpdmi
