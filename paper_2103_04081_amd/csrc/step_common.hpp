// Device pieces shared by the persistent step kernel and the grid-wide
// step kernels: the LDS region map, the CDF refresh of one mode (Section
// 3.1 distributions), Gs on the matrix cores, the step rules and the
// inverse-CDF search.
#pragma once

#include "cpd_internal.hpp"

namespace cpdmi {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

typedef uint32_t u4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// One chunk (U K-steps of 4 fibres) of the contraction of BF16-stored
// fibres, on v_mfma_f32_16x16x32_bf16 in K blocks of 32 fibres.  wa[u4][rt]
// holds the lane's WH values of K-steps 4 u4 .. 4 u4 + 3 (rank tile rt),
// x[u][v] the lane's fibre values (exact BF16 in FP32) of K-step u, as the
// v_mfma_f32_16x16x4f32 form takes them.  Slot i of lane group g of the
// BF16 instruction is the fibre of K-step 4 (2p + i/4) + i%4 of the same
// lane, so both operands come from those registers: the fibre values as
// they are, WH cut by truncation into three BF16 terms whose sum is the
// FP32 value exactly.  Every product is then exact in FP32 and the sums
// are FP32, at 3 x 16 instead of 8 x 32 matrix-core cycles per 32 fibres.
// hi and lo terms go to acc, mid terms to acc2.
template <int U, int RT, int VW>
__device__ __forceinline__ void mfma_wh_x_bf16(const f4 (&wa)[U / 4][RT], const float (&x)[U][VW],
                                               f4 (&acc)[RT][VW], f4 (&acc2)[RT][VW]) {
  static_assert(U % 8 == 0, "K blocks of 32 fibres");
#pragma unroll
  for (int p = 0; p < U / 8; ++p) {
    u4v bx[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        bx[v][q] = (__float_as_uint(x[8 * p + 2 * q][v]) >> 16) |
                   (__float_as_uint(x[8 * p + 2 * q + 1][v]) & 0xFFFF0000u);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      u4v ah, am, al;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t hb[2], mb[2], lb[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int i = 2 * q + e;
          const float w = wa[2 * p + i / 4][rt][i % 4];
          hb[e] = __float_as_uint(w) & 0xFFFF0000u;
          const float r1 = w - __uint_as_float(hb[e]);
          mb[e] = __float_as_uint(r1) & 0xFFFF0000u;
          lb[e] = __float_as_uint(r1 - __uint_as_float(mb[e]));
        }
        ah[q] = (hb[0] >> 16) | hb[1];
        am[q] = (mb[0] >> 16) | mb[1];
        al[q] = (lb[0] >> 16) | (lb[1] & 0xFFFF0000u);
      }
      const bf8v a_h = __builtin_bit_cast(bf8v, ah);
      const bf8v a_m = __builtin_bit_cast(bf8v, am);
      const bf8v a_l = __builtin_bit_cast(bf8v, al);
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        const bf8v b = __builtin_bit_cast(bf8v, bx[v]);
        acc[rt][v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h, b, acc[rt][v], 0, 0, 0);
        acc2[rt][v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_m, b, acc2[rt][v], 0, 0, 0);
        acc[rt][v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_l, b, acc[rt][v], 0, 0, 0);
      }
    }
  }
}

extern __shared__ __align__(16) unsigned char cpd_smem[];

// Offsets of the LDS regions of one workgroup.  Pointers are always formed
// from the LDS array itself so the compiler keeps them in the LDS address
// space (DS instructions) instead of generic pointers.
struct Smem {
  uint32_t o_cdf, o_idx, o_ratio, o_words, o_wf, o_rinv, o_rowoff, o_wht, o_gs, o_gsp, o_mbuf,
      o_gram, o_part, o_red, o_wts, o_misc, o_sbuf, o_fac;
  int rp16, bpad, ms, nd, nblk, has_sbuf, has_fac;
  __device__ double* cdf() const { return (double*)(cpd_smem + o_cdf); }
  __device__ int32_t* idx() const { return (int32_t*)(cpd_smem + o_idx); }        // [f][slot]
  __device__ double* ratio() const { return (double*)(cpd_smem + o_ratio); }      // [slot][f]
  __device__ uint64_t* words() const { return (uint64_t*)(cpd_smem + o_words); }  // Philox
  __device__ float* wf() const { return (float*)(cpd_smem + o_wf); }              // w_f
  __device__ float* rinv() const { return (float*)(cpd_smem + o_rinv); }          // 1 / w_f
  // byte offset of fibre f in copy n at rowb()[(f >> 4) * 16 + (f & 3) * 4 + ((f >> 2) & 3)]:
  // the offsets of K-steps 4q..4q+3 for one lane group are one 16-byte read
  __device__ uint32_t* rowb() const { return (uint32_t*)(cpd_smem + o_rowoff); }
  __device__ float* wht() const { return (float*)(cpd_smem + o_wht); }            // WH, A layout
  __device__ float* gs() const { return (float*)(cpd_smem + o_gs); }              // Gs [rp16]^2
  __device__ float* gsp() const { return (float*)(cpd_smem + o_gsp); }            // Gs partials
  __device__ float* mbuf() const { return (float*)(cpd_smem + o_mbuf); }          // rows [I_n][ms]
  __device__ float* sbuf() const { return (float*)(cpd_smem + o_sbuf); }          // S^(n) rows
  // resident factors: A^(k)(i, r) at fac()[(coff()[k] + i) * R + r]
  __device__ float* fac() const { return (float*)(cpd_smem + o_fac); }
  __device__ double* gram() const { return (double*)(cpd_smem + o_gram); }
  __device__ double* part() const { return (double*)(cpd_smem + o_part); }
  __device__ double* red() const { return (double*)(cpd_smem + o_red); }
  __device__ double* wts() const { return (double*)(cpd_smem + o_wts); }
  __device__ int32_t* misc() const { return (int32_t*)(cpd_smem + o_misc); }
  __device__ int32_t* coff() const { return misc() + 8; }  // CDF offset of each mode
};
// misc(): [1] error, [2] rank flag, [4] next-step Philox blocks generated

__device__ inline int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Waits for this wave's LDS traffic and orders it against later LDS reads
// of other lanes of the same wave.
__device__ inline void wave_lds_sync() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup"); }

// Position of (K-step k, rank tile rt, lane) in the A-operand layout: the
// four K-steps 4q..4q+3 of one lane are contiguous (one 16-byte LDS read).
__device__ inline int wht_index(int k, int rt, int lane, int RT) {
  return ((k >> 2) * RT + rt) * 256 + lane * 4 + (k & 3);
}

// 1 / d in FP64 from the hardware reciprocal and two Newton steps
// (r <- r + r (1 - d r)), each one doubling the correct bits.
__device__ inline double rcp_f64(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// L D L^T = G (L unit lower triangular) of the padded Gram G (16 x 16 in
// LDS, rows and columns past R zero, padded pivots one) by one wave,
// right-looking, lane r holding row r (its first NR entries): at pivot j the
// rows store their column-j entries, every lane reads the column back, and
// row r subtracts M_rj (M_cj / d_j) from its entries c in (j, NR).  Entries
// above the diagonal are updated too (never read: the stores and the
// write-back take c <= r), so the updates need no lane masks; no square
// roots, one reciprocal per pivot.  Writes L into G's lower triangle, 1 / d_j
// into dinv (one past R), and 1 into *flag if a pivot d_j falls below
// kRankTol of its diagonal.  A call of its own: inlined, its 64 registers of
// rows and column push the step kernel's other values into scratch.
template <int NR>
__device__ __noinline__ void ldl_wave(CPD_LDS double* G, CPD_LDS double* col, CPD_LDS double* dinv,
                                      int R, CPD_LDS int32_t* flag) {
  const int lane = threadIdx.x & 63;
  const int row = lane < NR ? lane : NR - 1;  // lanes past NR mirror the last row
  double g[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) g[k] = G[row * 16 + k];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    if (j < R) {
      if (lane < NR) col[lane] = g[j];
      wave_lds_sync();
      double cv[NR];
#pragma unroll
      for (int c = j; c < NR; ++c) cv[c] = col[c];
      const double d = cv[j];
      const double diag = G[j * 16 + j];
      const bool okj = d > kRankTol * diag && isfinite(d);
      ok = ok && okj;
      const double inv = rcp_f64(okj ? d : 1.0);
      const double mrj = g[j];
#pragma unroll
      for (int c = j + 1; c < NR; ++c) g[c] -= mrj * (cv[c] * inv);
      g[j] = lane == j ? 1.0 : mrj * inv;
      if (lane == 0) dinv[j] = inv;
      wave_lds_sync();  // the column is read before the next pivot's stores
    } else if (lane == 0) {
      dinv[j] = 1.0;
    }
  }
  if (lane < NR) {
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if (k <= lane) G[lane * 16 + k] = g[k];
  }
  if (lane == 0 && !ok) *flag = 1;
}

// ---------------------------------------------------------------------------
// Leverage scores l_i = a_i^T (A^T A)^{-1} a_i = sum_j y_j^2 / d_j with
// L D L^T = A^T A (FP64) and L y = a_i, of a mode with R <= 16, into wts();
// everything padded to 16 ranks: the Gram's rows and columns past R are zero
// and its padded pivots one, so L and D are the identity there.  LDS:
// gram() holds G (16 x 16, then L in its lower triangle), gram() + 256 the
// pivot column, gram() + 272 the 1 / d_j; part() the Gram partials
// (kGramParts x 256).  Returns CPD_E_RANK_DEFICIENT when a pivot falls below
// kRankTol of its diagonal.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int leverage_one_tile(const ChainDesc* dp, const Smem& S, int n,
                                                 const float* mb, int ms) {
  const int R = dp->R, In = dp->dims[n];
  const int lane = threadIdx.x & 63, wave = uniform_int(threadIdx.x >> 6);
  double* G = S.gram();
  double* col = G + 256;
  double* rinv = G + 272;
  double* part = S.part();
  double* w = S.wts();
  // G = A^T A on the FP64 matrix cores (v_mfma_f64_16x16x4f64): the A and B
  // operands are the same value, lane l holding a_{4s + l/16}(l % 16) for
  // K-step s; element q of lane l's result is G(4q + l/16, l % 16).  Wave
  // p < kGramParts sums the K-steps p, p + kGramParts, ...; the partials are
  // added in order (every kernel that refreshes a leverage CDF sums in this
  // order, so they all give the same bits).
  constexpr int kp = kGramParts;
  if (wave < kp) {
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    const int nks = (In + 3) >> 2;
    const int r = lane & 15;
    const int rc = r < R ? r : R - 1;  // loads stay in the rows; zeros are selected
#pragma unroll 4
    for (int s = wave; s < nks; s += kp) {
      const int i = 4 * s + (lane >> 4);
      const float v = mb[(i < In ? i : In - 1) * ms + rc];
      const double x = (i < In && r < R) ? (double)v : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) part[wave * 256 + (4 * q + (lane >> 4)) * 16 + r] = acc[q];
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    double g = 0.0;
    for (int p = 0; p < kp; ++p) g += part[p * 256 + threadIdx.x];
    const int rr = threadIdx.x >> 4, cc = threadIdx.x & 15;
    if (rr == cc && rr >= R) g = 1.0;
    G[threadIdx.x] = g;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    ldl_wave<16>(lmem(G), lmem(col), lmem(rinv), R, lmem(S.misc() + 2));
  }
  __syncthreads();
  const int err = S.misc()[2] ? CPD_E_RANK_DEFICIENT : 0;
  // l_i = sum_j y_j^2 / d_j with L y = a_i (forward substitution, one row
  // per thread, y in registers)
  for (int i = threadIdx.x; i < In; i += kBlock) {
    double y[16];
    double l = 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (j < R) {
        double v = (double)mb[i * ms + j];
#pragma unroll
        for (int k = 0; k < j; ++k) v -= G[j * 16 + k] * y[k];
        y[j] = v;
        l += (v * v) * rinv[j];
      } else {
        y[j] = 0.0;
      }
    }
    w[i] = l;
  }
  __syncthreads();
  return err;
}

// Euclidean weight of row i held in global memory: the sum over r (in
// order) of A(i, r)^2 in FP64, each square exact, as the LDS form below
// computes it, with the entries loaded sixteen at a time.
__device__ __forceinline__ double row_sq_global(const float* mb, int i, int ms, int R) {
  constexpr int kW = 16;
  double acc = 0.0;
  int r = 0;
  for (; r + kW <= R; r += kW) {
    float v[kW];
#pragma unroll
    for (int j = 0; j < kW; ++j) v[j] = mb[i * ms + r + j];
#pragma unroll
    for (int j = 0; j < kW; ++j) {
      const double a = (double)v[j];
      acc = acc + a * a;
    }
  }
  for (; r < R; ++r) {
    const double a = (double)mb[i * ms + r];
    acc = acc + a * a;  // a*a is exact in FP64 for an FP32 a
  }
  return acc;
}

// ---------------------------------------------------------------------------
// CDF of mode n from its factor rows (row i at mb[i * ms]): in LDS, or in
// global memory for GROWS (Euclidean and uniform sampling only).
// ---------------------------------------------------------------------------
template <int RT, bool GROWS = false>
__device__ __forceinline__ int refresh_cdf(const ChainDesc* dp, const Smem& S, int n,
                                           const float* mb, int ms) {
  const int R = dp->R, In = dp->dims[n];
  double* w = S.wts();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int err = 0;
  if constexpr (RT == 1) {
    if (dp->sampler == CPD_SAMPLER_LEVERAGE) err = leverage_one_tile(dp, S, n, mb, ms);
  }
  // leverage scores for 16 < R <= 64 (refused beyond; the forward solve keeps
  // a row in registers)
  if constexpr (RT > 1 && RT <= kMaxRankTiles) if (dp->sampler == CPD_SAMPLER_LEVERAGE) {
    // leverage scores l_i = ||L^{-1} a_i||^2 with L L^T = A^T A (FP64)
    double* G = S.gram();
    const int npairs = R * (R + 1) / 2;
    if (npairs <= kBlock) {
      // pairs x row chunks, partials summed in a fixed order
      int nch = kBlock / npairs;
      if (nch > In) nch = In;
      const int pr = threadIdx.x % npairs, ch = threadIdx.x / npairs;
      if (ch < nch) {
        int r = 0, rem = pr;
        while (rem >= R - r) {
          rem -= R - r;
          ++r;
        }
        const int c = r + rem;
        double acc0 = 0.0, acc1 = 0.0;
        int i = ch;
        for (; i + nch < In; i += 2 * nch) {
          acc0 += (double)mb[i * ms + r] * (double)mb[i * ms + c];
          acc1 += (double)mb[(i + nch) * ms + r] * (double)mb[(i + nch) * ms + c];
        }
        if (i < In) acc0 += (double)mb[i * ms + r] * (double)mb[i * ms + c];
        S.part()[ch * npairs + pr] = acc0 + acc1;
      }
      __syncthreads();
      for (int p = threadIdx.x; p < npairs; p += kBlock) {
        int r = 0, rem = p;
        while (rem >= R - r) {
          rem -= R - r;
          ++r;
        }
        const int c = r + rem;
        double acc = 0.0;
        for (int q = 0; q < nch; ++q) acc += S.part()[q * npairs + p];
        G[r * R + c] = acc;
        G[c * R + r] = acc;
      }
    } else {
      for (int p = threadIdx.x; p < npairs; p += kBlock) {
        int r = 0, rem = p;
        while (rem >= R - r) {
          rem -= R - r;
          ++r;
        }
        const int c = r + rem;
        double acc = 0.0;
        for (int i = 0; i < In; ++i) acc += (double)mb[i * ms + r] * (double)mb[i * ms + c];
        G[r * R + c] = acc;
        G[c * R + r] = acc;
      }
    }
    __syncthreads();
    // Cholesky by one wave (lane = row); the lower triangle of G becomes L
    if (threadIdx.x < 64) {
      bool ok = true;
      for (int j = 0; j < R; ++j) {
        double d = G[j * R + j];
        const double diag = d;
        for (int k = 0; k < j; ++k) d -= G[j * R + k] * G[j * R + k];
        const bool okj = d > kRankTol * diag && isfinite(d);
        ok = ok && okj;
        const double ljj = okj ? sqrt(d) : 1.0;
        const double inv = 1.0 / ljj;
        for (int i = j + 1 + lane; i < R; i += 64) {
          double v = G[i * R + j];
          for (int k = 0; k < j; ++k) v -= G[i * R + k] * G[j * R + k];
          G[i * R + j] = v * inv;
        }
        wave_lds_sync();
        if (lane == 0) G[j * R + j] = ljj;
        wave_lds_sync();
      }
      if (lane == 0 && !ok) S.misc()[2] = 1;
    }
    __syncthreads();
    if (S.misc()[2]) err = CPD_E_RANK_DEFICIENT;
    // l_i by forward substitution L y = a_i (y in registers)
    for (int i = threadIdx.x; i < In; i += kBlock) {
      double y[RT * 16];
      double l = 0.0;
#pragma unroll
      for (int j = 0; j < RT * 16; ++j) {
        if (j < R) {
          double v = (double)mb[i * ms + j];
#pragma unroll
          for (int k = 0; k < j; ++k) v -= G[j * R + k] * y[k];
          y[j] = v / G[j * R + j];
          l += y[j] * y[j];
        } else {
          y[j] = 0.0;
        }
      }
      w[i] = l;
    }
    __syncthreads();
  }
  // quantise: q_i = ceil(w_i 2^E), 2^E * max(w) * 2^ceil(log2 In) < 2^53,
  // then the inclusive prefix sum (exact integers, so any order gives the
  // same bits)
  double* red = S.red();
  double* C = S.cdf() + S.coff()[n];
  CPD_GLOBAL double* Cg = gmem(dp->C[n]);
  const int c = bit_length_u32((uint32_t)(In - 1));
  if (In <= kBlock) {
    const int i = threadIdx.x;
    double wi = 0.0;
    if (i < In) {
      if (dp->sampler == CPD_SAMPLER_EUCLIDEAN) {
        if constexpr (GROWS) {
          wi = row_sq_global(mb, i, ms, R);
        } else {
          for (int r = 0; r < R; ++r) {
            const double a = (double)mb[i * ms + r];
            wi = wi + a * a;  // a*a is exact in FP64 for an FP32 a
          }
        }
      } else if (dp->sampler == CPD_SAMPLER_UNIFORM) {
        wi = 1.0;
      } else {
        wi = w[i];
      }
    }
    const bool fin = i >= In || (isfinite(wi) && wi >= 0.0);
    double m = fin ? wi : __builtin_inf();
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if (lane == 0) red[wave] = m;
    __syncthreads();
    double wmax = red[0];
    for (int j = 1; j < kWaves; ++j) wmax = fmax(wmax, red[j]);
    if (!(wmax > 0.0) || !isfinite(wmax)) return err ? err : CPD_E_DEGENERATE;
    int ex;
    frexp(wmax, &ex);
    double q = i < In ? ceil(ldexp(wi, 52 - ex - c)) : 0.0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double u = __shfl_up(q, o);
      if (lane >= o) q += u;
    }
    if (lane == 63) red[kWaves + wave] = q;
    __syncthreads();
    double off = 0.0;
    for (int j = 0; j < wave; ++j) off += red[kWaves + j];
    if (i < In) {
      C[i] = q + off;
      Cg[i] = q + off;
    }
    return err;
  }
  // general path (more rows than threads)
  if (dp->sampler != CPD_SAMPLER_LEVERAGE) {
    for (int i = threadIdx.x; i < In; i += kBlock) {
      double acc = 0.0;
      if (dp->sampler == CPD_SAMPLER_EUCLIDEAN) {
        if constexpr (GROWS) {
          acc = row_sq_global(mb, i, ms, R);
        } else {
          for (int r = 0; r < R; ++r) {
            const double a = (double)mb[i * ms + r];
            acc = acc + a * a;
          }
        }
      } else {
        acc = 1.0;
      }
      w[i] = acc;
    }
  }
  double m = 0.0;
  for (int i = threadIdx.x; i < In; i += kBlock)
    m = fmax(m, (isfinite(w[i]) && w[i] >= 0.0) ? w[i] : __builtin_inf());
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  __syncthreads();
  if (lane == 0) red[wave] = m;
  __syncthreads();
  double wmax = red[0];
  for (int j = 1; j < kWaves; ++j) wmax = fmax(wmax, red[j]);
  if (!(wmax > 0.0) || !isfinite(wmax)) return err ? err : CPD_E_DEGENERATE;
  int ex;
  frexp(wmax, &ex);
  double carry = 0.0;
  for (int base = 0; base < In; base += kBlock) {
    const int i = base + threadIdx.x;
    double q = i < In ? ceil(ldexp(w[i], 52 - ex - c)) : 0.0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double u = __shfl_up(q, o);
      if (lane >= o) q += u;
    }
    __syncthreads();
    if (lane == 63) red[kWaves + wave] = q;
    __syncthreads();
    double off = carry, tot = carry;
    for (int j = 0; j < kWaves; ++j) {
      if (j < wave) off += red[kWaves + j];
      tot += red[kWaves + j];
    }
    if (i < In) {
      C[i] = q + off;
      Cg[i] = q + off;
    }
    carry = tot;
  }
  return err;
}

// ---------------------------------------------------------------------------
// Gs = (WH)^T H, 16x16 tiles, the K-steps split over the waves; partial
// tiles summed in a fixed order.  H = WH / w is recovered in the B operand.
//   A operand (16 x 4): lane l holds WH[f0 + l/16][rt*16 + l%16]
//   B operand (4 x 16): lane l holds H[f0 + l/16][ct*16 + l%16]
//   D (16 x 16): lane l, element q holds row 4*(l/16)+q, column l%16
// Gs rows are rp16 + GPAD floats apart in LDS.
// ---------------------------------------------------------------------------
template <int RT, int NT = kBlock, int GPAD = 0>
__device__ __forceinline__ void compute_gs(const Smem& S) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = uniform_int(threadIdx.x >> 6);
  const int fl = lane >> 4, cl = lane & 15;
  constexpr int T2 = RT * RT;
  constexpr int kparts = T2 >= NW ? 1 : NW / T2;
  constexpr int items = T2 * kparts;
  const int nq = S.bpad / 16;  // groups of four K-steps
  const float* wht = S.wht();
  const float* rinv = S.rinv();
  float* gsp = S.gsp();
  if constexpr (T2 >= 2 * NW && NW % RT == 0) {
    // several whole tiles per wave, all in the wave's column tile
    // ct = wave % RT: the H operand is formed once per K group and up to
    // four tiles accumulate side by side (independent matrix-core chains),
    // each in the same order as one tile alone
    constexpr int M = T2 / NW;
    constexpr int MB = M < 4 ? M : 4;
    const int ct = wave % RT;
    for (int m0 = 0; m0 < M; m0 += MB) {
      f4 g[MB];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) g[mb] = f4{0.f, 0.f, 0.f, 0.f};
      for (int q = 0; q < nq; ++q) {
        const f4 h4 = *(const f4*)(wht + (q * RT + ct) * 256 + lane * 4);
        float b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = h4[j] * rinv[(4 * q + j) * 4 + fl];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const int rt = (wave + NW * (m0 + mb)) / RT;
          const f4 a4 = *(const f4*)(wht + (q * RT + rt) * 256 + lane * 4);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            g[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[j], b[j], g[mb], 0, 0, 0);
        }
      }
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int rt = (wave + NW * (m0 + mb)) / RT;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          S.gs()[(rt * 16 + 4 * fl + e) * (S.rp16 + GPAD) + ct * 16 + cl] = g[mb][e];
      }
    }
    __syncthreads();
    return;
  }
  for (int it = wave; it < items; it += NW) {
    const int tile = it % T2, kp = it / T2;
    const int rt = tile / RT, ct = tile % RT;
    const int q0 = kp * nq / kparts, q1 = (kp + 1) * nq / kparts;
    f4 g = f4{0.f, 0.f, 0.f, 0.f};
    for (int q = q0; q < q1; ++q) {
      const f4 a4 = *(const f4*)(wht + (q * RT + rt) * 256 + lane * 4);
      const f4 h4 = *(const f4*)(wht + (q * RT + ct) * 256 + lane * 4);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float b = h4[j] * rinv[(4 * q + j) * 4 + fl];
        g = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[j], b, g, 0, 0, 0);
      }
    }
    if constexpr (kparts == 1) {
      // one part per tile: straight to Gs
#pragma unroll
      for (int e = 0; e < 4; ++e)
        S.gs()[(rt * 16 + 4 * fl + e) * (S.rp16 + GPAD) + ct * 16 + cl] = g[e];
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) gsp[it * 256 + (4 * fl + e) * 16 + cl] = g[e];
    }
  }
  __syncthreads();
  if constexpr (kparts == 1) return;
  const int rp16 = S.rp16;
  for (int e = threadIdx.x; e < rp16 * rp16; e += NT) {
    const int r = e / rp16, s2 = e - r * rp16;
    const int tile = (r >> 4) * RT + (s2 >> 4);
    float acc = 0.f;
    for (int kp = 0; kp < kparts; ++kp)
      acc += gsp[(kp * T2 + tile) * 256 + (r & 15) * 16 + (s2 & 15)];
    S.gs()[r * (rp16 + GPAD) + s2] = acc;
  }
  __syncthreads();
}

// A uniform value kept in a vector register: the compiler may not re-load it
// from the descriptor (a scalar load and a full wait) every time it is used.
template <typename T>
__device__ __forceinline__ T in_vgpr(T x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Step-rule parameters of one step, held in vector registers.
struct UpdateParams {
  float alpha_t, eta, b;
  int ada, nonneg;
};

__device__ __forceinline__ UpdateParams update_params(const ChainDesc* dp, uint64_t t) {
  UpdateParams u;
  u.alpha_t = in_vgpr(dp->rule == CPD_RULE_DECREASING
                          ? (float)(dp->beta / ((double)t + dp->gamma))
                          : dp->alpha);
  u.eta = in_vgpr(dp->eta);
  u.b = in_vgpr(dp->b);
  u.ada = in_vgpr((int)(dp->rule == CPD_RULE_ADAGRAD));
  u.nonneg = in_vgpr(dp->nonneg);
  return u;
}

// The update of one entry: returns the new value, updates the accumulator.
__device__ __forceinline__ float update_entry(const UpdateParams& u, float a, float g,
                                              float& sacc) {
  float an;
  if (u.ada) {
    sacc = sacc + g * g;
    const float d2 = u.b + sacc;
    // eta g / sqrt(b + S) with the hardware reciprocal square root (1 ulp)
    an = d2 > 0.f ? a - u.eta * g * __builtin_amdgcn_rsqf(d2) : a;
  } else {
    an = a - u.alpha_t * g;
  }
  if (u.nonneg) an = fmaxf(an, 0.f);
  return an;
}


// first i in [0, Ik) with C[i] > tg (C ascending, C[Ik-1] > tg)
__device__ inline int cdf_search(const double* C, int Ik, double tg) {
  int pos = 0;
  for (int len = 1 << (31 - __clz(Ik)); len > 0; len >>= 1)
    if (pos + len <= Ik && C[pos + len - 1] <= tg) pos += len;
  return pos < Ik ? pos : Ik - 1;
}


}  // namespace cpdmi
