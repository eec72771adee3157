// Persistent step kernel: one 1024-thread workgroup advances one
// decomposition by many SGD steps without leaving the chip.
//
// One step (paper Section 3, Algorithms 3-5):
//   1. mode draw and inverse-CDF sampling of B rows per mode k != n from the
//      integer-valued CDFs held in LDS (Philox4x64-10 words, Lemmas 2/4);
//   2. p_f = prod_k q_k(i_k)/Q_k, w_f = 1/(B p_f), fibre row offsets by the
//      unfolding index map, sampled KRP rows H (Hadamard of factor rows);
//   3. Gs = H^T W H in FP64, then WH in place;
//   4. M^T = (WH)^T X_s on the matrix cores (v_mfma_f32_16x16x4f32): every
//      wave owns a 16-column tile of the I_n x R output and streams the
//      gathered fibres straight from HBM into the B operand; the fibre dimension
//      is split across waves when there are fewer than 16 tiles and the partial
//      tiles are summed in a fixed order;
//   5. G = A^(n) Gs - M and the fixed / decreasing / AdaGrad update;
//   6. the CDF of mode n is rebuilt from the new factor (squared row norms or
//      leverage scores via FP64 Gram + Cholesky), quantised to exact integers.
#include "cpd_internal.hpp"

namespace cpdmi {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Block-wide maximum (every thread receives it).  scratch: kWaves doubles.
__device__ double block_max(double v, double* scratch) {
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = scratch[0];
  for (int i = 1; i < kWaves; ++i) r = fmax(r, scratch[i]);
  return r;
}

// In-place inclusive prefix sum of data[0..L) in LDS.  The values are
// integers below 2^53, so every partial sum is exact and the order of the
// additions does not matter.  scratch: kWaves doubles.
__device__ void block_scan(double* data, int L, double* scratch) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double carry = 0.0;
  for (int base = 0; base < L; base += kBlock) {
    const int i = base + threadIdx.x;
    double v = i < L ? data[i] : 0.0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double u = __shfl_up(v, o);
      if (lane >= o) v += u;
    }
    __syncthreads();
    if (lane == 63) scratch[w] = v;
    __syncthreads();
    double off = carry, tot = carry;
    for (int j = 0; j < kWaves; ++j) {
      if (j < w) off += scratch[j];
      tot += scratch[j];
    }
    if (i < L) data[i] = v + off;
    carry = tot;
  }
  __syncthreads();
}

__device__ inline void pair_of(int pr, int R, int& r, int& s) {
  int rr = 0;
  while (pr >= R - rr) {
    pr -= R - rr;
    ++rr;
  }
  r = rr;
  s = rr + pr;
}

// Symmetric Gram-type sum out[r][s] = sum_{e < n} x(e, r) x(e, s) * wt(e), FP64,
// for the R(R+1)/2 pairs, summed in a fixed order.  `get(e, r)` returns a
// double; `wt(e)` the weight.  part: >= kBlock doubles.
template <typename Get, typename Wt>
__device__ void gram_fixed_order(int n, int R, Get get, Wt wt, double* out, double* part) {
  const int npairs = R * (R + 1) / 2;
  if (npairs <= kBlock) {
    int nch = kBlock / npairs;
    if (nch > n) nch = n;
    if (nch < 1) nch = 1;
    const int pr = threadIdx.x % npairs, ch = threadIdx.x / npairs;
    if (ch < nch) {
      int r, s;
      pair_of(pr, R, r, s);
      double acc = 0.0;
      for (int e = ch; e < n; e += nch) acc += wt(e) * (get(e, r) * get(e, s));
      part[ch * npairs + pr] = acc;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < npairs; p += kBlock) {
      int r, s;
      pair_of(p, R, r, s);
      double acc = 0.0;
      for (int c = 0; c < nch; ++c) acc += part[c * npairs + p];
      out[r * R + s] = acc;
      out[s * R + r] = acc;
    }
  } else {
    for (int p = threadIdx.x; p < npairs; p += kBlock) {
      int r, s;
      pair_of(p, R, r, s);
      double acc = 0.0;
      for (int e = 0; e < n; ++e) acc += wt(e) * (get(e, r) * get(e, s));
      out[r * R + s] = acc;
      out[s * R + r] = acc;
    }
  }
  __syncthreads();
}

struct Smem {
  double* cdf;
  int32_t* idx;
  uint64_t* words;
  double* wf;
  int64_t* rowoff;
  float* hb;
  double* gs;
  float* mbuf;
  double* part;
  double* wts;
  int32_t* misc;  // [0] mode, [1] error, [2..] scratch
  double* red;    // kWaves doubles for reductions
  int* coff;      // LDS: offset of each mode's CDF
  int rp16, bpad, ms, nd;
};

// Rebuild the integer-valued CDF of mode n from the factor rows held in
// mbuf (row i at mbuf[i * ms], R floats).  Returns a cpd_status.
__device__ int refresh_cdf(const ChainDesc* dp, Smem& S, int n) {
  const int R = dp->R, In = dp->dims[n];
  const int ms = S.ms;
  double* w = S.wts;
  int err = 0;
  if (dp->sampler == CPD_SAMPLER_UNIFORM) {
    for (int i = threadIdx.x; i < In; i += kBlock) w[i] = 1.0;
  } else if (dp->sampler == CPD_SAMPLER_EUCLIDEAN) {
    for (int i = threadIdx.x; i < In; i += kBlock) {
      double acc = 0.0;
      for (int r = 0; r < R; ++r) {
        const double a = (double)S.mbuf[i * ms + r];
        acc = acc + a * a;  // a*a is exact in FP64 for an FP32 a
      }
      w[i] = acc;
    }
  } else {
    // leverage scores: l_i = ||L^{-1} a_i||^2 with L L^T = A^T A (FP64)
    double* G = S.gs;           // R x R, becomes L (lower triangle)
    double* Li = S.part;        // R x R, L^{-1} (lower triangle)
    const float* mb = S.mbuf;
    gram_fixed_order(
        In, R, [&](int e, int r) { return (double)mb[e * ms + r]; }, [](int) { return 1.0; }, G,
        S.part);
    if (threadIdx.x == 0) S.misc[2] = 0;
    __syncthreads();
    for (int j = 0; j < R; ++j) {
      // every thread reads the same pivot, so the branch below is uniform
      double d = G[j * R + j];
      const double diag = d;
      for (int k = 0; k < j; ++k) d -= G[j * R + k] * G[j * R + k];
      const bool ok = d > kRankTol * diag && isfinite(d);
      const double ljj = ok ? sqrt(d) : 1.0;
      __syncthreads();
      if (threadIdx.x == 0) {
        G[j * R + j] = ljj;
        if (!ok) S.misc[2] = 1;
      }
      for (int i = j + 1 + (int)threadIdx.x; i < R; i += kBlock) {
        double v = G[i * R + j];
        for (int k = 0; k < j; ++k) v -= G[i * R + k] * G[j * R + k];
        G[i * R + j] = v / ljj;
      }
      __syncthreads();
    }
    if (S.misc[2]) err = CPD_E_RANK_DEFICIENT;
    // columns of L^{-1}, one lane per column
    for (int c = threadIdx.x; c < R; c += kBlock) {
      for (int j = 0; j < R; ++j) {
        if (j < c) {
          Li[j * R + c] = 0.0;
          continue;
        }
        double v = j == c ? 1.0 : 0.0;
        for (int k = c; k < j; ++k) v -= G[j * R + k] * Li[k * R + c];
        Li[j * R + c] = v / G[j * R + j];
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < In; i += kBlock) {
      double l = 0.0;
      for (int j = 0; j < R; ++j) {
        double y = 0.0;
        for (int k = 0; k <= j; ++k) y += Li[j * R + k] * (double)mb[i * ms + k];
        l += y * y;
      }
      w[i] = l;
    }
  }
  __syncthreads();
  // quantise: q_i = ceil(w_i 2^E), 2^E * max(w) * 2^ceil(log2 In) < 2^53
  double lmax = 0.0;
  bool fin = true;
  for (int i = threadIdx.x; i < In; i += kBlock) {
    lmax = fmax(lmax, w[i]);
    fin = fin && isfinite(w[i]) && w[i] >= 0.0;
  }
  if (!fin) S.misc[3] = 1;
  const double wmax = block_max(lmax, S.red);
  const bool bad = S.misc[3] != 0;
  __syncthreads();
  if (bad || !(wmax > 0.0) || !isfinite(wmax)) {
    if (threadIdx.x == 0) S.misc[3] = 0;
    __syncthreads();
    return err ? err : CPD_E_DEGENERATE;
  }
  int ex;
  frexp(wmax, &ex);
  const int c = bit_length_u32((uint32_t)(In - 1));
  const int E = 52 - ex - c;
  double* C = S.cdf + S.coff[n];
  for (int i = threadIdx.x; i < In; i += kBlock) C[i] = ceil(ldexp(w[i], E));
  __syncthreads();
  block_scan(C, In, S.red);
  double* Cg = dp->C[n];
  for (int i = threadIdx.x; i < In; i += kBlock) Cg[i] = C[i];
  __syncthreads();
  return err;
}

// ---------------------------------------------------------------------------
// The contraction M^T (R x I_n) = (WH)^T (R x B) * X_s (B x I_n) for one
// column tile, K = fibres [4*k0, 4*k1).  VW consecutive columns per lane
// (one MFMA per column slot), RT row tiles of 16.
//   A operand (16 x 4): lane l holds WH[f0 + l/16][rt*16 + l%16]
//   B operand (4 x 16): lane l holds X_s[f0 + l/16][col + (l%16)*VW + v]
//   D (16 x 16): lane l, element q holds row 4*(l/16)+q, column l%16
// ---------------------------------------------------------------------------
template <int VW, int RT, bool BF16, int U>
__device__ void contract_tile(f4 (&acc)[RT][VW], const void* __restrict__ Xn,
                              const int64_t* __restrict__ rowoff, const float* __restrict__ wh,
                              int rp16, int col0, int k0, int k1) {
  const int lane = threadIdx.x & 63;
  const int fl = lane >> 4, cl = lane & 15;
  const int col = col0 + cl * VW;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int v = 0; v < VW; ++v) acc[rt][v] = f4{0.f, 0.f, 0.f, 0.f};

  // two register buffers with compile-time indices (a runtime-indexed
  // private array would live in scratch memory)
  float xa[U][VW], xb[U][VW];
  auto load = [&](float (&x)[U][VW], int kbase) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ks = kbase + u;
      if (ks < k1) {
        const int f = ks * 4 + fl;
        const int64_t off = rowoff[f] + col;
        if constexpr (BF16) {
          const uint32_t pk = *(const uint32_t*)((const uint16_t*)Xn + off);
          x[u][0] = __uint_as_float(pk << 16);
          if constexpr (VW > 1) x[u][1] = __uint_as_float(pk & 0xFFFF0000u);
        } else {
          const float* p = (const float*)Xn + off;
#pragma unroll
          for (int v = 0; v < VW; ++v) x[u][v] = p[v];
        }
      } else {
#pragma unroll
        for (int v = 0; v < VW; ++v) x[u][v] = 0.f;
      }
    }
  };
  auto compute = [&](const float (&x)[U][VW], int kbase) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ks = kbase + u;
      if (ks < k1) {
        const int f = ks * 4 + fl;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          const float a = wh[f * rp16 + rt * 16 + cl];
#pragma unroll
          for (int v = 0; v < VW; ++v)
            acc[rt][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, x[u][v], acc[rt][v], 0, 0, 0);
        }
      }
    }
  };
  if (k0 >= k1) return;
  load(xa, k0);
  for (int kb = k0; kb < k1; kb += 2 * U) {
    if (kb + U < k1) load(xb, kb + U);
    compute(xa, kb);
    if (kb + 2 * U < k1) load(xa, kb + 2 * U);
    if (kb + U < k1) compute(xb, kb + U);
  }
}

template <int VW, int RT>
__device__ void store_tile(const f4 (&acc)[RT][VW], float* mbuf, int ms, int R, int In, int col0,
                           bool add) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int v = 0; v < VW; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = rt * 16 + 4 * (lane >> 4) + q;
        const int i = col0 + (lane & 15) * VW + v;
        if (r < R && i < In) {
          float* m = mbuf + i * ms + r;
          *m = add ? *m + acc[rt][v][q] : acc[rt][v][q];
        }
      }
}

template <int VW, int RT, bool BF16>
__device__ void contraction(const ChainDesc* dp, Smem& S, int n) {
  constexpr int U = (VW * RT <= 2) ? 16 : 8;
  const int In = dp->dims[n];
  const int SW = 16 * VW;
  const int nst = (In + SW - 1) / SW;
  const int ks = dp->ksplit[n];
  const int KS = S.bpad / 4;
  const int wave = threadIdx.x >> 6;
  f4 acc[RT][VW];
  if (ks <= 1) {
    for (int st = wave; st < nst; st += kWaves) {
      contract_tile<VW, RT, BF16, U>(acc, dp->X[n], S.rowoff, S.hb, S.rp16, st * SW, 0, KS);
      store_tile<VW, RT>(acc, S.mbuf, S.ms, dp->R, In, st * SW, false);
    }
    __syncthreads();
  } else {
    const bool has = wave < nst * ks;
    const int st = wave % nst, kc = wave / nst;
    if (has) {
      const int k0 = (int)((int64_t)kc * KS / ks), k1 = (int)((int64_t)(kc + 1) * KS / ks);
      contract_tile<VW, RT, BF16, U>(acc, dp->X[n], S.rowoff, S.hb, S.rp16, st * SW, k0, k1);
    }
    for (int round = 0; round < ks; ++round) {
      if (has && kc == round) store_tile<VW, RT>(acc, S.mbuf, S.ms, dp->R, In, st * SW, round > 0);
      __syncthreads();
    }
  }
}

template <int VW, bool BF16>
__device__ void contraction_rt(const ChainDesc* dp, Smem& S, int n) {
  switch (dp->RT) {
    case 1: contraction<VW, 1, BF16>(dp, S, n); break;
    case 2: contraction<VW, 2, BF16>(dp, S, n); break;
    case 3: contraction<VW, 3, BF16>(dp, S, n); break;
    default: contraction<VW, 4, BF16>(dp, S, n); break;
  }
}

__global__ void __launch_bounds__(kBlock) chain_kernel(const ChainDesc* __restrict__ descs,
                                                       StepArgs args) {
  extern __shared__ __align__(16) unsigned char smem[];
  const ChainDesc* dp = descs + blockIdx.x;
  if (!dp->active) return;
  ChainState* st = dp->state;
  if (args.op != OP_SAMPLE && args.op != OP_REFRESH && st->status != 0) return;
  const int tid = threadIdx.x;
  const int N = dp->N, R = dp->R, B = dp->B;
  const LdsPlan P = lds_plan(N, dp->dims, R, B);
  Smem S;
  S.cdf = (double*)(smem + P.cdf);
  S.idx = (int32_t*)(smem + P.idx);
  S.words = (uint64_t*)(smem + P.words);
  S.wf = (double*)(smem + P.wf);
  S.rowoff = (int64_t*)(smem + P.rowoff);
  S.hb = (float*)(smem + P.hb);
  S.gs = (double*)(smem + P.gs);
  S.mbuf = (float*)(smem + P.mbuf);
  S.part = (double*)(smem + P.part);
  S.wts = (double*)(smem + P.wts);
  S.misc = (int32_t*)(smem + P.misc);
  S.red = (double*)(smem + P.red);
  S.rp16 = P.rp16;
  S.bpad = P.bpad;
  S.ms = P.ms;
  S.nd = P.nd;
  S.coff = S.misc + 8;
  if (tid < 8) S.misc[tid] = 0;
  if (tid == 0) {
    int o = 0;
    for (int k = 0; k < N; ++k) {
      S.coff[k] = o;
      o += dp->dims[k];
    }
  }
  __syncthreads();
  for (int k = 0; k < N; ++k)
    for (int i = tid; i < dp->dims[k]; i += kBlock) S.cdf[S.coff[k] + i] = dp->C[k][i];
  __syncthreads();

  if (args.op == OP_REFRESH) {
    int err = 0;
    for (int n = 0; n < N && !err; ++n) {
      for (int e = tid; e < dp->dims[n] * R; e += kBlock) {
        const int i = e / R, r = e - i * R;
        S.mbuf[i * S.ms + r] = dp->A[n][e];
      }
      __syncthreads();
      err = refresh_cdf(dp, S, n);
    }
    if (tid == 0 && err) st->status = err;
    return;
  }

  const int64_t t0 = args.op == OP_SAMPLE ? (int64_t)args.sample_t : st->t;
  int64_t nsteps = args.op == OP_STEP ? args.nsteps : 1;
  if (args.op == OP_STEP && dp->step_limit > 0 && t0 + nsteps > dp->step_limit)
    nsteps = dp->step_limit > t0 ? dp->step_limit - t0 : 0;
  const int nm1 = N - 1;
  const int nd = S.nd;
  int64_t done = 0;
  int err = 0;

  for (int64_t s = 0; s < nsteps; ++s) {
    const uint64_t t = (uint64_t)(t0 + s);
    // ---- 1. draws -------------------------------------------------------
    if (args.op == OP_REPLAY) {
      // caller-supplied indices: reject any outside its mode's range
      for (int e = tid; e < B * nm1; e += kBlock) {
        const int sl = e % nm1;
        const int k = sl < args.replay_mode ? sl : sl + 1;
        const int i = args.replay_idx[e];
        if (i < 0 || i >= dp->dims[k]) S.misc[1] = CPD_E_INVALID;
        S.idx[e] = i < 0 ? 0 : (i >= dp->dims[k] ? dp->dims[k] - 1 : i);
      }
    } else {
      const int nblk = (nd + 3) / 4;
      for (int b = tid; b < nblk; b += kBlock) {
        uint64_t o[4];
        philox4x64_10(t, (uint64_t)b, 0, 0, dp->key0, dp->key1, o);
        S.words[4 * b + 0] = o[0];
        S.words[4 * b + 1] = o[1];
        S.words[4 * b + 2] = o[2];
        S.words[4 * b + 3] = o[3];
      }
    }
    __syncthreads();
    if (S.misc[1]) {
      err = S.misc[1];
      break;
    }
    const int n = args.op == OP_REPLAY ? args.replay_mode : (int)mulhi_u64(S.words[0], (uint64_t)N);
    double* ratio = (double*)S.words;
    for (int d = 1 + tid; d < nd; d += kBlock) {
      const int sl = (d - 1) / B, f = (d - 1) - sl * B;
      const int k = sl < n ? sl : sl + 1;
      const double* Ck = S.cdf + S.coff[k];
      const int Ik = dp->dims[k];
      const double Q = Ck[Ik - 1];
      int i;
      if (args.op == OP_REPLAY) {
        i = S.idx[f * nm1 + sl];
      } else {
        const double tg = (double)mulhi_u64(S.words[d], (uint64_t)Q);
        int lo = 0, hi = Ik - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (Ck[mid] > tg) hi = mid;
          else lo = mid + 1;
        }
        i = lo;
        S.idx[f * nm1 + sl] = i;
      }
      const double q = Ck[i] - (i ? Ck[i - 1] : 0.0);
      ratio[d] = q / Q;
    }
    __syncthreads();
    // ---- 2. probabilities, weights, fibre rows, KRP rows ----------------
    const int ldn = dp->ld[n];
    for (int f = tid; f < S.bpad; f += kBlock) {
      if (f < B) {
        double p = 1.0;
        int64_t j = 0, stride = 1;
        int sl = 0;
        for (int k = 0; k < N; ++k) {
          if (k == n) continue;
          p = p * ratio[1 + sl * B + f];
          j += (int64_t)S.idx[f * nm1 + sl] * stride;
          stride *= dp->dims[k];
          ++sl;
        }
        S.wf[f] = 1.0 / ((double)B * p);
        S.rowoff[f] = j * ldn;
        if (args.op == OP_SAMPLE) {
          args.out_p[f] = p;
          for (int q = 0; q < nm1; ++q) args.out_idx[f * nm1 + q] = S.idx[f * nm1 + q];
        }
      } else {
        S.wf[f] = 0.0;
        S.rowoff[f] = 0;
      }
    }
    if (args.op == OP_SAMPLE) {
      if (tid == 0) *args.out_mode = n;
      return;
    }
    for (int e = tid; e < S.bpad * S.rp16; e += kBlock) {
      const int f = e / S.rp16, r = e - f * S.rp16;
      float h = 0.f;
      if (f < B && r < R) {
        int sl = 0;
        bool first = true;
        for (int k = 0; k < N; ++k) {
          if (k == n) continue;
          const float a = dp->A[k][(int64_t)S.idx[f * nm1 + sl] * R + r];
          h = first ? a : h * a;
          first = false;
          ++sl;
        }
      }
      S.hb[e] = h;
    }
    __syncthreads();
    // ---- 3. Gs = H^T W H (FP64), then WH in place ------------------------
    {
      const float* hb = S.hb;
      const double* wf = S.wf;
      const int rp = S.rp16;
      gram_fixed_order(
          B, R, [&](int f, int r) { return (double)hb[f * rp + r]; },
          [&](int f) { return wf[f]; }, S.gs, S.part);
    }
    for (int e = tid; e < S.bpad * S.rp16; e += kBlock) {
      const int f = e / S.rp16;
      S.hb[e] = (float)(S.wf[f] * (double)S.hb[e]);
    }
    __syncthreads();
    // ---- 4. M^T = (WH)^T X_s on the matrix cores -------------------------
    if (dp->dtype == CPD_BF16) contraction_rt<2, true>(dp, S, n);
    else contraction_rt<1, false>(dp, S, n);
    // ---- 5. G = A Gs - M and the update -----------------------------------
    const int In = dp->dims[n];
    float* An = dp->A[n];
    float* Sn = dp->S[n];
    const double alpha_t =
        dp->rule == CPD_RULE_DECREASING ? dp->beta / ((double)t + dp->gamma) : (double)dp->alpha;
    bool bad = false;
    for (int e = tid; e < In * R; e += kBlock) {
      const int i = e / R, r = e - i * R;
      const float* arow = An + (int64_t)i * R;
      double ag = 0.0;
      for (int q = 0; q < R; ++q) ag += (double)arow[q] * S.gs[q * R + r];
      const float g = (float)(ag - (double)S.mbuf[i * S.ms + r]);
      const float a = arow[r];
      float an;
      if (dp->rule == CPD_RULE_ADAGRAD) {
        const float acc = Sn[e] + g * g;
        Sn[e] = acc;
        const float den = sqrtf(dp->b + acc);
        an = den > 0.f ? a - dp->eta * g / den : a;
      } else {
        an = a - (float)alpha_t * g;
      }
      if (dp->nonneg) an = fmaxf(an, 0.f);
      if (!isfinite(an)) bad = true;
      S.mbuf[i * S.ms + r] = an;
    }
    if (bad) S.misc[1] = CPD_E_DIVERGED;
    __syncthreads();
    for (int e = tid; e < In * R; e += kBlock) {
      const int i = e / R, r = e - i * R;
      An[e] = S.mbuf[i * S.ms + r];
    }
    ++done;
    if (S.misc[1]) {
      err = S.misc[1];
      break;
    }
    // ---- 6. distribution of mode n from the new factor -------------------
    if (dp->sampler != CPD_SAMPLER_UNIFORM) {
      err = refresh_cdf(dp, S, n);
      if (err) break;
    }
  }
  if (tid == 0) {
    if (args.op == OP_STEP || args.op == OP_REPLAY) st->t = t0 + done;
    if (err) st->status = err;
  }
}

// Host-side launcher (declared in cpd_runtime.hpp).
hipError_t launch_chain_kernel(const ChainDesc* descs, int nchains, size_t lds_bytes,
                               const StepArgs& args, hipStream_t stream) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)chain_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(chain_kernel, dim3(nchains), dim3(kBlock), lds_bytes, stream, descs, args);
  return hipGetLastError();
}

}  // namespace cpdmi
