// Grid-wide SGD step for mini-batches too large for one workgroup.  The
// step is the same as the persistent kernel's (paper Section 3, Algorithms
// 3-5; the same Philox words, integer CDFs, draws and step rules), spread
// over the whole GPU in three launches:
//   wide_gather_kernel   every block takes a slice of the B sampled fibres
//                        (with few slices, several blocks share a slice
//                        and split its row tiles):
//                        the Philox blocks of its draws, inverse-CDF search
//                        over the CDFs in LDS, p_f, w_f and the WH rows, its
//                        part of Gs = (WH)^T H, then its part of
//                        -G^T = (WH)^T X_s - Gs A^(n)T on the matrix cores
//                        (v_mfma_f32_16x16x4f32, fibres streamed from HBM
//                        into the B operand), written to HBM;
//   wide_update_kernel   sums the block parts of every entry of A^(n) in a
//                        fixed order and applies the step rule;
//   wide_refresh_kernel  the CDF of the updated mode (squared row norms or
//                        leverage scores), the same code as the persistent
//                        kernel's refresh.
// G = A^(n) Gs - M is linear in the fibres, so the block parts add up to the
// gradient of eq. (gradient); only the FP32 summation order differs from
// the persistent kernel.
#include "cpd_runtime.hpp"
#include "step_common.hpp"

namespace cpdmi {

constexpr int kUpdWaves = 16;    // waves of an update block
constexpr int kUpdEntries = 16;  // entries of A^(n) per update block

template <int RT, bool BF16>
__global__ void __launch_bounds__(kGatherThreads) wide_gather_kernel(const ChainDesc* __restrict__ dp,
                                                             WideArgs a) {
  ChainState* st = dp->state;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = uniform_int(tid >> 6);
  const int fl = lane >> 4, cl = lane & 15;
  const int N = dp->N, R = dp->R, B = dp->B, nm1 = N - 1;
  const int FB = a.fb;
  // block tb of slice `slice` (a.tsplit blocks per slice)
  const int slice = blockIdx.x / a.tsplit, tb = blockIdx.x - slice * a.tsplit;
  const int f0 = slice * FB;
  const int nf = B - f0 < FB ? B - f0 : FB;
  const GatherPlan P = gather_plan(N, dp->dims, RT, FB);
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
  S.o_misc = P.misc;
  S.o_mbuf = S.o_gram = S.o_part = S.o_red = S.o_wts = S.o_sbuf = S.o_fac = 0;
  S.rp16 = 16 * RT;
  S.bpad = (int)round_up(nf, kFibrePad);
  S.ms = S.nd = S.nblk = S.has_sbuf = S.has_fac = 0;
  int32_t* misc = S.misc();
  const int64_t t = a.op == OP_SAMPLE ? (int64_t)a.sample_t : st->t;
  // One phase before the first barrier: the first CDF values are loaded into
  // registers, the Philox blocks of this slice's draws (which do not depend
  // on the mode) are computed while they are in flight, then the values are
  // stored.  The last thread draws the mode and reads the sticky status
  // (misc: [0] stop, [1] error, [3] mode), so the whole block agrees on them.
  int sumdims = 0;
  for (int k = 0; k < N; ++k) sumdims += dp->dims[k];
  auto cdf_at = [&](int e) {
    int k = 0, o = 0;
    while (e >= o + dp->dims[k]) o += dp->dims[k++];
    return gmem(dp->C[k])[e - o];
  };
  constexpr int kCdfRegs = 4;
  double cv[kCdfRegs];
#pragma unroll
  for (int j = 0; j < kCdfRegs; ++j) {
    const int e = tid + j * kGatherThreads;
    cv[j] = e < sumdims ? cdf_at(e) : 0.0;
  }
  uint64_t* words = S.words();
  const int nwb = P.nwb;
  if (a.op != OP_REPLAY) {
    // draw d = 1 + slot * B + f uses word d % 4 of the Philox block (t, d / 4)
    for (int e = tid; e < nm1 * nwb; e += kGatherThreads) {
      const int sl = e / nwb, j = e - sl * nwb;
      const int64_t dfirst = 1 + (int64_t)sl * B + f0;
      const int64_t c = (dfirst >> 2) + j;
      if (c <= ((dfirst + nf - 1) >> 2)) {
        uint64_t o[4];
        philox4x64_10((uint64_t)t, (uint64_t)c, 0, 0, dp->key0, dp->key1, o);
        words[4 * e + 0] = o[0];
        words[4 * e + 1] = o[1];
        words[4 * e + 2] = o[2];
        words[4 * e + 3] = o[3];
      }
    }
  }
  if (tid == kGatherThreads - 1) {
    misc[0] = a.op != OP_SAMPLE && st->status != 0;
    misc[1] = 0;
    int o = 0;
    for (int k = 0; k < N; ++k) {
      S.coff()[k] = o;
      o += dp->dims[k];
    }
    int nd;
    if (a.op == OP_REPLAY) {
      nd = a.replay_mode;
    } else if (a.force_mode1) {
      nd = a.force_mode1 - 1;
    } else {
      uint64_t w0[4];
      philox4x64_10((uint64_t)t, 0, 0, 0, dp->key0, dp->key1, w0);
      nd = (int)mulhi_u64(w0[0], (uint64_t)N);
    }
    misc[3] = nd;
  }
  // the CDFs of all modes, back to back in mode order
#pragma unroll
  for (int j = 0; j < kCdfRegs; ++j) {
    const int e = tid + j * kGatherThreads;
    if (e < sumdims) S.cdf()[e] = cv[j];
  }
  for (int e = tid + kCdfRegs * kGatherThreads; e < sumdims; e += kGatherThreads) S.cdf()[e] = cdf_at(e);
  __syncthreads();
  if (misc[0]) return;
  const int n = uniform_int(misc[3]);
  for (int e = tid; e < nm1 * nf; e += kGatherThreads) {
    const int sl = e / nf, f = e - sl * nf;
    const int k = sl < n ? sl : sl + 1;
    const double* Ck = S.cdf() + S.coff()[k];
    const int Ik = dp->dims[k];
    const double Q = Ck[Ik - 1];
    int i;
    if (a.op == OP_REPLAY) {
      // caller-supplied indices: reject any outside its mode's range
      i = gmem(a.replay_idx)[(int64_t)(f0 + f) * nm1 + sl];
      if (i < 0 || i >= Ik) {
        misc[1] = CPD_E_INVALID;
        i = 0;
      }
    } else {
      const int64_t dfirst = 1 + (int64_t)sl * B + f0;
      const int64_t d = dfirst + f;
      const uint64_t wd = words[4 * (sl * nwb + (int)((d >> 2) - (dfirst >> 2))) + (int)(d & 3)];
      i = cdf_search(Ck, Ik, (double)mulhi_u64(wd, (uint64_t)Q));
    }
    S.idx()[f * nm1 + sl] = i;
    S.ratio()[sl * FB + f] = (Ck[i] - (i ? Ck[i - 1] : 0.0)) / Q;
  }
  __syncthreads();
  if (misc[1]) {
    if (tid == 0) st->status = misc[1];
    return;
  }
  // ---- per fibre: p_f, w_f, the fibre's byte offset in copy n -------------
  const int ldn = dp->ld[n];
  const int64_t esz = BF16 ? 2 : 4;
  for (int f = tid; f < S.bpad; f += kGatherThreads) {
    const int ro = (f >> 4) * 16 + (f & 3) * 4 + ((f >> 2) & 3);
    if (f < nf) {
      double p = 1.0;
      int64_t j = 0, stride = 1;
      int sl = 0;
      for (int k = 0; k < N; ++k) {
        if (k == n) continue;
        p = p * S.ratio()[sl * FB + f];
        j += (int64_t)S.idx()[f * nm1 + sl] * stride;
        stride *= dp->dims[k];
        ++sl;
      }
      S.wf()[f] = (float)(1.0 / ((double)B * p));
      S.rinv()[f] = (float)((double)B * p);
      S.rowb()[ro] = (uint32_t)(j * ldn * esz);
      if (a.op == OP_SAMPLE && tb == 0) {
        gmem(a.out_p)[f0 + f] = p;
        for (int q = 0; q < nm1; ++q)
          gmem(a.out_idx)[(int64_t)(f0 + f) * nm1 + q] = S.idx()[f * nm1 + q];
      }
    } else {
      S.wf()[f] = 0.f;
      S.rinv()[f] = 0.f;
      S.rowb()[ro] = 0;
    }
  }
  if (a.op == OP_SAMPLE) {
    if (blockIdx.x == 0 && tid == 0) *gmem(a.out_mode) = n;
    return;
  }
  // ---- WH rows: H(f, c) = product over k != n (ascending) of A^(k)(i_k, c),
  // scaled by w_f (the same expression as above), four columns per item, in
  // the A-operand order of the matrix-core instruction ----------------------
  float* wht = S.wht();
  {
    constexpr int CPI = 4, ipf = 16 * RT / CPI;
    for (int itm = tid; itm < S.bpad * ipf; itm += kGatherThreads) {
      const int f = itm / ipf, c0 = (itm - f * ipf) * CPI;
      float h[CPI];
#pragma unroll
      for (int c = 0; c < CPI; ++c) h[c] = 0.f;
      float wfl = 0.f;
      if (f < nf) {
        double p = 1.0;
        for (int sl = 0; sl < nm1; ++sl) p = p * S.ratio()[sl * FB + f];
        wfl = (float)(1.0 / ((double)B * p));
        for (int q = 0; q < nm1; ++q) {
          const int k = q < n ? q : q + 1;
          const CPD_GLOBAL float* row = gmem(dp->A[k]) + (int64_t)S.idx()[f * nm1 + q] * R;
#pragma unroll
          for (int c = 0; c < CPI; ++c) {
            const float v = c0 + c < R ? row[c0 + c] : 0.f;
            h[c] = q == 0 ? v : h[c] * v;
          }
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
  if (blockIdx.x == 0 && tid == 0) {
    a.info->t = t;
    a.info->n = n;
  }
  // ---- this slice's -G^T, per 16-column tile of the I_n x R output ---------
  //   A operand: lane l holds WH[f0 + l/16][rt*16 + l%16]           (LDS)
  //   B operand: lane l holds X_s[f0 + l/16][col0 + (l%16)*VW + v]   (HBM)
  // then K = rank with A = -Gs[rt*16 + l%16][s] and B = A^(n)[col][s],
  // s = 4 kk + l/16 at step kk (kk + 4 RT (l/16) from four rank tiles).
  constexpr int VW = BF16 ? 2 : 1;
  constexpr int U = chunk_steps(VW, RT);  // K-steps per chunk
  constexpr bool kGsVec = RT >= 4;        // the epilogue's Gs entries in 16-byte reads
  const int In = dp->dims[n];
  const int SW = 16 * VW;
  const int nst = (In + SW - 1) / SW;
  const int nck = S.bpad / (4 * U);
  // wave w owns tiles tg, tg + tgs, ... of its tile group (tile group
  // tg = tb * 8/kp + w % (8/kp) of the slice's tgs = tsplit * 8/kp) and
  // walks each over its part of the slice's fibres (long runs of loads in
  // flight per wave measured faster than walking the tiles chunk by chunk).
  // Every block splits its chunks as a full slice would, so the part count
  // is the same for all slices; waves of a short last slice may get no chunk.
  const int nck_full = FB / (4 * U);
  const int kp = wide_kparts(nst, nck_full);
  const int tgn = kGatherWaves / kp;
  const int kpart = wave / tgn;
  const int tg = tb * tgn + wave % tgn, tgs = a.tsplit * tgn;
  const int c0 = kpart * nck_full / kp;
  const int c1 = min((kpart + 1) * nck_full / kp, nck);
  const int nckw = c1 > c0 ? c1 - c0 : 0;
  const int nitems = tg < nst ? (nst - 1 - tg) / tgs + 1 : 0;
  const float* __restrict__ whtc = S.wht();
  const uint32_t* __restrict__ rowb = S.rowb();
  const CPD_GLOBAL char* __restrict__ Xb = gmem((const char*)dp->X[n]);
  const CPD_GLOBAL float* An = gmem(dp->A[n]);
  CPD_GLOBAL float* part = gmem(a.part) + ((int64_t)slice * kp + kpart) * R * In;
  const int rp16 = S.rp16;

  f4 acc[RT][VW], acc2[RT][VW];
  // two register buffers of fibre values, each with the A^(n) entries of the
  // -Gs A^(n)T term, loaded with the last chunk of a tile
  float xbuf[kGatherBufs][U][VW];
  float pbuf[kGatherBufs][4 * RT][VW];
  auto load = [&](float (&x)[U][VW], float (&pA)[4 * RT][VW], int c) {
    const int it = c / nckw;
    const int stl = tg + it * tgs;
    const int ci = c0 + (c - it * nckw);
    const int kq0 = ci * (U / 4);  // first group of four K-steps
    const uint32_t colb = (uint32_t)((stl * SW + cl * VW) * (BF16 ? 2 : 4));
#pragma unroll
    for (int u4 = 0; u4 < U / 4; ++u4) {
      const uint4 ob = *(const uint4*)(rowb + (kq0 + u4) * 16 + fl * 4);
      const uint32_t o4[4] = {ob.x, ob.y, ob.z, ob.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const CPD_GLOBAL char* p = Xb + (o4[j] + colb);
        const int u = 4 * u4 + j;
        if constexpr (BF16) {
          const uint32_t pk = *(const CPD_GLOBAL uint32_t*)p;
          x[u][0] = __uint_as_float(pk << 16);
          x[u][VW - 1] = __uint_as_float(pk & 0xFFFF0000u);
        } else {
          x[u][0] = *(const CPD_GLOBAL float*)p;
        }
      }
    }
    if (ci == c1 - 1) {
      // rank columns past R and rows past I_n read as zero (the first part
      // adds the term)
      const int col0 = stl * SW;
#pragma unroll
      for (int kk = 0; kk < 4 * RT; ++kk) {
        const int s = kGsVec ? kk + 4 * RT * fl : 4 * kk + fl;  // K slot fl of step kk
#pragma unroll
        for (int v = 0; v < VW; ++v) {
          const int i = col0 + cl * VW + v;
          pA[kk][v] = (kpart == 0 && s < R && i < In) ? An[(int64_t)i * R + s] : 0.f;
        }
      }
    }
  };
  auto epilogue = [&](int stl, const float (&pA)[4 * RT][VW]) {
    const int col0 = stl * SW;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < VW; ++v) acc[rt][v] += acc2[rt][v];
    if constexpr (!kGsVec) {
#pragma unroll
      for (int kk = 0; kk < 4 * RT; ++kk) {
        const int s = 4 * kk + fl;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          const float g = -S.gs()[(rt * 16 + cl) * (rp16 + kGsPad) + s];
#pragma unroll
          for (int v = 0; v < VW; ++v)
            acc[rt][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(g, pA[kk][v], acc[rt][v], 0, 0, 0);
        }
      }
    } else {
      // four or more rank tiles: step kk, slot fl is rank s = kk + 4 RT fl,
      // so a lane's Gs entries of four consecutive steps are one 16-byte LDS
      // read (rank tiles four at a time: at most four reads in registers)
#pragma unroll
      for (int kk4 = 0; kk4 < RT; ++kk4)
#pragma unroll
        for (int r0 = 0; r0 < RT; r0 += 4) {
          f4 g4[4];
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (r0 + r < RT)
              g4[r] = *(const f4*)(S.gs() + ((r0 + r) * 16 + cl) * (rp16 + kGsPad) +
                                   4 * RT * fl + 4 * kk4);
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (r0 + r < RT)
#pragma unroll
                for (int v = 0; v < VW; ++v)
                  acc[r0 + r][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                      -g4[r][j], pA[4 * kk4 + j][v], acc[r0 + r][v], 0, 0, 0);
        }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int v = 0; v < VW; ++v)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = rt * 16 + 4 * fl + q;
          const int i = col0 + cl * VW + v;
          if (r < R && i < In) part[(int64_t)r * In + i] = acc[rt][v][q];
        }
  };
  auto compute = [&](const float (&x)[U][VW], const float (&pA)[4 * RT][VW], int c) {
    const int it = c / nckw;
    const int ci = c0 + (c - it * nckw);
    const int kq0 = ci * (U / 4);
    if (ci == c0) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int v = 0; v < VW; ++v) {
          acc[rt][v] = f4{0.f, 0.f, 0.f, 0.f};
          acc2[rt][v] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    f4 wa[U / 4][RT];
#pragma unroll
    for (int u4 = 0; u4 < U / 4; ++u4)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        wa[u4][rt] = *(const f4*)(whtc + ((kq0 + u4) * RT + rt) * 256 + lane * 4);
    if constexpr (BF16 && U % 8 == 0) {
      mfma_wh_x_bf16<U, RT, VW>(wa, x, acc, acc2);
    } else {
#pragma unroll
      for (int u4 = 0; u4 < U / 4; ++u4)
#pragma unroll
        for (int j = 0; j < 4; j += 2)
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int v = 0; v < VW; ++v) {
              acc[rt][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[u4][rt][j], x[4 * u4 + j][v],
                                                                acc[rt][v], 0, 0, 0);
              acc2[rt][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                  wa[u4][rt][j + 1], x[4 * u4 + j + 1][v], acc2[rt][v], 0, 0, 0);
            }
    }
    if (ci == c1 - 1) epilogue(tg + it * tgs, pA);
  };
  const int total = nitems * nckw;
  if (nitems > 0 && nckw == 0) {
    // a short last block: this part of every tile of the wave is zero
    for (int it = 0; it < nitems; ++it) {
      const int col0 = (tg + it * tgs) * SW;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int v = 0; v < VW; ++v)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = rt * 16 + 4 * fl + q;
            const int i = col0 + cl * VW + v;
            if (r < R && i < In) part[(int64_t)r * In + i] = 0.f;
          }
    }
  }
  __syncthreads();
  // the first chunks' fibre loads are in flight while this slice's Gs forms;
  // then the loads of the next kGatherBufs - 1 chunks while one is multiplied
#pragma unroll
  for (int j = 0; j < kGatherBufs - 1; ++j)
    if (j < total) load(xbuf[j], pbuf[j], j);
  compute_gs<RT, kGatherThreads, kGsPad>(S);
  for (int c = 0; c < total; c += kGatherBufs) {
#pragma unroll
    for (int j = 0; j < kGatherBufs; ++j) {
      constexpr int kNb = kGatherBufs;
      if (c + j + kNb - 1 < total)
        load(xbuf[(j + kNb - 1) % kNb], pbuf[(j + kNb - 1) % kNb], c + j + kNb - 1);
      if (c + j < total) compute(xbuf[j], pbuf[j], c + j);
    }
  }
}

// Entry e = r * I_n + i of -G^T: the block parts summed in a fixed order,
// then the step rule on A^(n)(i, r).  A block takes 16 entries; its 64 lane
// groups of 16 lanes (four per wave) sum the parts g, g + 64, g + 128, ...
// (one 64-byte row segment per part and lane group), then one thread per
// entry adds the 64 group sums in order.
__global__ void __launch_bounds__(64 * kUpdWaves) wide_update_kernel(
    const ChainDesc* __restrict__ dp, const float* __restrict__ part, int nblocks, int fb,
    const WideInfo* __restrict__ info) {
  constexpr int kGroups = 4 * kUpdWaves;
  static_assert(kUpdEntries == 16, "one entry per lane of a 16-lane group");
  __shared__ float red[kGroups][kUpdEntries + 1];
  __shared__ int sh_stop, sh_n;
  __shared__ int64_t sh_t;
  ChainState* st = dp->state;
  if (threadIdx.x == 0) {
    sh_stop = st->status != 0;
    sh_n = info->n;
    sh_t = info->t;
  }
  __syncthreads();
  if (sh_stop) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = wave * 4 + (lane >> 4), ec = lane & 15;
  const int n = sh_n;
  const int64_t t = sh_t;
  const int In = dp->dims[n], R = dp->R, E = In * R;
  // the parts the gather kernel wrote: wide_kparts of the mode per block
  const int vw = dp->dtype == CPD_BF16 ? 2 : 1;
  const int nparts =
      nblocks * wide_kparts((In + 16 * vw - 1) / (16 * vw), fb / (4 * chunk_steps(vw, dp->RT)));
  const int e = blockIdx.x * kUpdEntries + ec;
  // the entry this thread updates: its A and S values are loaded with the
  // parts
  const int e1 = blockIdx.x * kUpdEntries + (int)threadIdx.x;
  const bool upd = threadIdx.x < kUpdEntries && e1 < E;
  const int64_t ai = upd ? (int64_t)(e1 % In) * R + e1 / In : 0;
  CPD_GLOBAL float* An = gmem(dp->A[n]);
  CPD_GLOBAL float* Sn = gmem(dp->S[n]);
  const UpdateParams up = update_params(dp, (uint64_t)t);
  const float a_old = upd ? An[ai] : 0.f;
  float sacc = (upd && up.ada) ? Sn[ai] : 0.f;
  float s = 0.f;
  if (e < E) {
    const CPD_GLOBAL float* pp = gmem(part) + e;
    int b = g;
    for (; b + 7 * kGroups < nparts; b += 8 * kGroups) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = pp[(int64_t)(b + j * kGroups) * E];
#pragma unroll
      for (int j = 0; j < 8; ++j) s = s + v[j];
    }
    for (; b < nparts; b += kGroups) s = s + pp[(int64_t)b * E];
  }
  red[g][ec] = s;
  __syncthreads();
  if (upd) {
    float m = red[0][threadIdx.x];
    for (int q = 1; q < kGroups; ++q) m = m + red[q][threadIdx.x];
    const float an = update_entry(up, a_old, -m, sacc);
    if (up.ada) Sn[ai] = sacc;
    An[ai] = an;
    if (!isfinite(an)) st->status = CPD_E_DIVERGED;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st->t = t + 1;
}

// The same update when every entry has at most kGroups parts (few slices):
// one thread per entry, the parts added in the order and with the zero
// terms of wide_update_kernel's group sums, so the result is the same bits.
constexpr int kUpdFewThreads = 256;
__global__ void __launch_bounds__(kUpdFewThreads) wide_update_few_kernel(
    const ChainDesc* __restrict__ dp, const float* __restrict__ part, int nblocks, int fb,
    const WideInfo* __restrict__ info) {
  constexpr int kGroups = 4 * kUpdWaves;
  ChainState* st = dp->state;
  const int n = info->n;
  const int64_t t = info->t;
  if (st->status != 0) return;
  const int In = dp->dims[n], R = dp->R, E = In * R;
  const int vw = dp->dtype == CPD_BF16 ? 2 : 1;
  const int nparts =
      nblocks * wide_kparts((In + 16 * vw - 1) / (16 * vw), fb / (4 * chunk_steps(vw, dp->RT)));
  const int e = blockIdx.x * kUpdFewThreads + (int)threadIdx.x;
  if (e < E) {
    const int64_t ai = (int64_t)(e % In) * R + e / In;
    CPD_GLOBAL float* An = gmem(dp->A[n]);
    CPD_GLOBAL float* Sn = gmem(dp->S[n]);
    const UpdateParams up = update_params(dp, (uint64_t)t);
    const float a_old = An[ai];
    float sacc = up.ada ? Sn[ai] : 0.f;
    const CPD_GLOBAL float* pp = gmem(part) + e;
    float m = 0.f + pp[0];
    for (int q = 1; q < nparts; ++q) m = m + (0.f + pp[(int64_t)q * E]);
    if (nparts < kGroups) m = m + 0.f;
    const float an = update_entry(up, a_old, -m, sacc);
    if (up.ada) Sn[ai] = sacc;
    An[ai] = an;
    if (!isfinite(an)) st->status = CPD_E_DIVERGED;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st->t = t + 1;
}

// CDF of one mode (mode >= 0), of every mode (-1, one block per mode) or of
// the mode of the step in flight (-2, after its update).
template <int RT>
__global__ void __launch_bounds__(kBlock) wide_refresh_kernel(const ChainDesc* __restrict__ dp,
                                                              const WideInfo* __restrict__ info,
                                                              int mode) {
  ChainState* st = dp->state;
  // status and mode loaded together (one round trip)
  const int32_t status = st->status;
  const int ninfo = mode == -2 ? info->n : 0;
  if (mode == -2 && status != 0) return;
  const int tid = threadIdx.x;
  const int N = dp->N, R = dp->R;
  const RefreshPlan P = refresh_plan(N, dp->dims, R, RT);
  Smem S;
  S.o_cdf = P.cdf;
  S.o_mbuf = P.mbuf;
  S.o_gram = P.gram;
  S.o_part = P.part;
  S.o_red = P.red;
  S.o_wts = P.wts;
  S.o_misc = P.misc;
  S.o_idx = S.o_ratio = S.o_words = S.o_wf = S.o_rinv = S.o_rowoff = S.o_wht = S.o_gs =
      S.o_gsp = S.o_sbuf = S.o_fac = 0;
  S.ms = P.ms;
  S.rp16 = 16 * RT;
  S.bpad = S.nd = S.nblk = S.has_sbuf = S.has_fac = 0;
  // every mode's CDF goes to the same LDS region (offset 0)
  if (tid < 8 + kMaxModes) S.misc()[tid] = 0;
  float* mbuf = S.mbuf();
  // mode -1: one block per mode
  const int nb = mode >= 0 ? mode : (mode == -1 ? (int)blockIdx.x : ninfo);
  const int ne = nb + 1;
  int err = 0;
  for (int n = nb; n < ne && !err; ++n) {
    const CPD_GLOBAL float* An = gmem(dp->A[n]);
    if (P.rows_in_lds) {
      for (int e = tid; e < dp->dims[n] * R; e += kBlock) {
        const int i = e / R;
        mbuf[i * P.ms + (e - i * R)] = An[e];
      }
      __syncthreads();
      err = refresh_cdf<RT>(dp, S, n, S.mbuf(), S.ms);
    } else {
      // rows too large for LDS: the squared row norms from global memory
      err = refresh_cdf<RT, true>(dp, S, n, dp->A[n], R);
    }
    __syncthreads();
  }
  if (tid == 0 && err) st->status = err;
}

template <int RT, bool BF16>
static hipError_t gather_attr() {
  static std::atomic<uint32_t> attr_set{0};
  return set_lds_limit_once((const void*)wide_gather_kernel<RT, BF16>, 160 * 1024, &attr_set);
}

template <int RT>
static hipError_t refresh_attr() {
  static std::atomic<uint32_t> attr_set{0};
  return set_lds_limit_once((const void*)wide_refresh_kernel<RT>, 160 * 1024, &attr_set);
}

template <int RT>
static hipError_t prepare_rt(int dtype) {
  hipError_t e = dtype == CPD_BF16 ? gather_attr<RT, true>() : gather_attr<RT, false>();
  return e == hipSuccess ? refresh_attr<RT>() : e;
}

hipError_t prepare_wide_kernels(int rt, int dtype) {
  switch (rt) {
    case 1: return prepare_rt<1>(dtype);
    case 2: return prepare_rt<2>(dtype);
    case 3: return prepare_rt<3>(dtype);
    case 4: return prepare_rt<4>(dtype);
    default: return prepare_rt<kWideRt>(dtype);
  }
}

template <int RT, bool BF16>
static hipError_t gather_rt(const ChainDesc* d, int nblocks, size_t lds, const WideArgs& a,
                            hipStream_t s) {
  hipError_t e = gather_attr<RT, BF16>();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((wide_gather_kernel<RT, BF16>), dim3(nblocks * a.tsplit), dim3(kGatherThreads),
                     lds, s, d, a);
  return hipGetLastError();
}

hipError_t launch_wide_gather(const ChainDesc* d_desc, int rt, int dtype, int nblocks,
                              size_t lds_bytes, const WideArgs& a, hipStream_t stream) {
  const bool bf = dtype == CPD_BF16;
  switch (rt) {
    case 1: return bf ? gather_rt<1, true>(d_desc, nblocks, lds_bytes, a, stream)
                      : gather_rt<1, false>(d_desc, nblocks, lds_bytes, a, stream);
    case 2: return bf ? gather_rt<2, true>(d_desc, nblocks, lds_bytes, a, stream)
                      : gather_rt<2, false>(d_desc, nblocks, lds_bytes, a, stream);
    case 3: return bf ? gather_rt<3, true>(d_desc, nblocks, lds_bytes, a, stream)
                      : gather_rt<3, false>(d_desc, nblocks, lds_bytes, a, stream);
    case 4: return bf ? gather_rt<4, true>(d_desc, nblocks, lds_bytes, a, stream)
                      : gather_rt<4, false>(d_desc, nblocks, lds_bytes, a, stream);
    default: return bf ? gather_rt<kWideRt, true>(d_desc, nblocks, lds_bytes, a, stream)
                       : gather_rt<kWideRt, false>(d_desc, nblocks, lds_bytes, a, stream);
  }
}

hipError_t launch_wide_update(const ChainDesc* d_desc, const float* part, int nblocks, int fb,
                              const WideInfo* info, int max_entries, hipStream_t stream) {
  if (nblocks * kWideMaxParts <= 4 * kUpdWaves) {
    // at most 4 * kUpdWaves parts per entry whatever the mode
    const int grid = (max_entries + kUpdFewThreads - 1) / kUpdFewThreads;
    hipLaunchKernelGGL(wide_update_few_kernel, dim3(grid), dim3(kUpdFewThreads), 0, stream,
                       d_desc, part, nblocks, fb, info);
    return hipGetLastError();
  }
  const int grid = (max_entries + kUpdEntries - 1) / kUpdEntries;
  hipLaunchKernelGGL(wide_update_kernel, dim3(grid), dim3(64 * kUpdWaves), 0, stream, d_desc,
                     part, nblocks, fb, info);
  return hipGetLastError();
}

template <int RT>
static hipError_t refresh_rt(const ChainDesc* d, size_t lds, const WideInfo* info, int mode,
                             int nmodes, hipStream_t s) {
  hipError_t e = refresh_attr<RT>();
  if (e != hipSuccess) return e;
  const int grid = mode == -1 ? nmodes : 1;
  hipLaunchKernelGGL(wide_refresh_kernel<RT>, dim3(grid), dim3(kBlock), lds, s, d, info, mode);
  return hipGetLastError();
}

hipError_t launch_wide_refresh(const ChainDesc* d_desc, int rt, size_t lds_bytes,
                               const WideInfo* info, int mode, int nmodes, hipStream_t stream) {
  if (mode == -1 && (nmodes < 1 || nmodes > kMaxModes)) return hipErrorInvalidValue;
  switch (rt) {
    case 1: return refresh_rt<1>(d_desc, lds_bytes, info, mode, nmodes, stream);
    case 2: return refresh_rt<2>(d_desc, lds_bytes, info, mode, nmodes, stream);
    case 3: return refresh_rt<3>(d_desc, lds_bytes, info, mode, nmodes, stream);
    case 4: return refresh_rt<4>(d_desc, lds_bytes, info, mode, nmodes, stream);
    default: return refresh_rt<kWideRt>(d_desc, lds_bytes, info, mode, nmodes, stream);
  }
}

}  // namespace cpdmi
