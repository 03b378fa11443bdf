// Free-space particle-particle translations (Section 4.2, Graf's addition
// theorem), evaluated directly for every pair.
//
// Incoming coefficients of the target m collect from every source l != m
//   a^m_i += sum_j t_{i-j} alpha^l_j,  t_nu = H_nu(k |x_m - x_l|) e^{-i nu (th_ml - pi)},
// with th_ml the polar angle of x_m - x_l, k = kp for alpha and ks for beta.
// The adjoint (conjugate transpose) maps target-side vectors back to the
// sources with conj(t_{-nu}).
//
// Right-hand sides are taken RB at a time by one workgroup: the symbols of a
// partner batch are built once and applied to each of them.
//
// One workgroup of 2 ROWS lanes per output particle (ROWS = 32 for orders up
// to 15, 64 for order 16): lanes [0, ROWS) own the P modes, [ROWS, 2 ROWS)
// the S modes of that particle.  Partners are taken 16 at a
// time; 32 lanes build the 16 x 2 Toeplitz symbols in LDS (Hankel functions
// by forward recurrence from H_0, H_1, stable because |Y_nu| dominates), then
// every lane runs its row of the Toeplitz product against the partner
// coefficients staged in LDS.  With tabulated symbols and one right-hand side
// each lane instead takes one partner of a batch of 4 and 4 adjacent rows,
// sliding the symbol entries through registers (one LDS read of the symbol
// per four complex multiply-adds): 0.64 -> 0.47 ms (FP64) and 0.49 -> 0.37
// ms (mixed) at 20000 particles, order 15.
#include "dev.h"
#include "ems_internal.h"
#include "graf_sym.h"

namespace ems {

template <bool MIXED> struct CT;
template <> struct CT<false> {
  using T = double2;
  __device__ static T from(double2 v) { return v; }
};
template <> struct CT<true> {
  using T = float2;
  __device__ static T from(double2 v) { return make_float2((float)v.x, (float)v.y); }
};

__device__ __forceinline__ void cfma_any(double2 &a, double2 x, double2 y) { cfma(a, x, y); }
__device__ __forceinline__ void cfma_any(float2 &a, float2 x, float2 y) { cfmaf(a, x, y); }
__device__ __forceinline__ double2 conj_any(double2 v) { return make_double2(v.x, -v.y); }
// the tabulated near-pair symbols are read once per apply: non-temporal
// loads keep them from displacing the partner coefficients in the caches
typedef double graf_d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 sym_load(const double2 *p) {
  const graf_d2v v = __builtin_nontemporal_load(reinterpret_cast<const graf_d2v *>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 conj_any(float2 v) { return make_float2(v.x, -v.y); }

// ADJ: the adjoint map (a compile-time choice, so the inner products carry no
// per-element branch); the tabulated symbols serve only the forward map.
template <int PM, bool MIXED, int RB, bool STORED, bool ADJ>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(STORED && RB == 1 ? 3 : 1))) void graf_direct_kernel(
    int n, int nrhs, const double *__restrict__ xy, const int *__restrict__ p,
    const int64_t *__restrict__ off, const double2 *__restrict__ x, int64_t ldx,
    double2 *__restrict__ out, int64_t ldo, double kp, double ks, int adjoint,
    const int *__restrict__ nbr_ptr, const int *__restrict__ nbr_idx,
    const double2 *__restrict__ nsym, const int64_t *__restrict__ nbr_off,
    const int *__restrict__ nbr_p) {
  static_assert(!(STORED && ADJ), "tabulated near-field symbols are forward only");
  (void)adjoint;
  using T = typename CT<MIXED>::T;
  constexpr int NT = 4 * PM + 1;
  constexpr int NM = 2 * PM + 1;
  // partners per batch: generated symbols amortise the Hankel work over 16;
  // tabulated ones are only copied, and a small batch keeps LDS low enough
  // for several wavefronts per CU to hide the loads
  constexpr int SB = STORED ? 4 : 16;
  constexpr int ROWS = 2 * PM + 1 <= 32 ? 32 : 64;
  __shared__ T t_lds[2][SB][NT];
  __shared__ T c_lds[SB][2][NM];

  const int b = blockIdx.x;
  const int r0 = blockIdx.y * RB;  // right-hand sides r0 .. r0 + RB - 1 share the symbols
  const int lane = threadIdx.x;
  const double bx = xy[2 * b], by = xy[2 * b + 1];
  const int pb = p[b];
  const int w = lane / ROWS;
  const int i = lane % ROWS - PM;
  T acc[RB];
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
    acc[rr].x = 0;
    acc[rr].y = 0;
  }
  // partners: every other particle, or the near list of b
  const int np = nbr_ptr ? nbr_ptr[b + 1] - nbr_ptr[b] : n;
  const int *nl = nbr_ptr ? nbr_idx + nbr_ptr[b] : nullptr;

  if constexpr (STORED && RB == 1) {
    // Software-pipelined form of the tabulated near field, one right-hand
    // side: while batch k is multiplied out of LDS, the symbols and partner
    // coefficients of batch k+1 are in flight into registers, and the
    // partner offsets of batch k+2 (read by pair position) behind them, so
    // no global-load chain is waited for between batches.
    constexpr int TH = 2 * ROWS;
    constexpr int NSY = SB * 2 * NT, NCF = SB * 2 * NM;
    constexpr int PS = (NSY + TH - 1) / TH, PC = (NCF + TH - 1) / TH;
    const int pb0 = nbr_ptr[b];
    const double2 *xr = x + (int64_t)r0 * ldx;
    int64_t po[PC];
    int pp[PC];
    double2 rs[PS], rc[PC];
    // Products: lane (hq, rq) of its wave type's ROWS lanes takes partner hq
    // of each batch and rows i0 .. i0 + kR - 1.  Row i0 + k needs at
    // coefficient jj the symbol entry that row i0 needs at jj - k, so the
    // entries slide through a window of kR registers: one symbol read from
    // LDS per kR complex multiply-adds (the LDS reads bound the one-row-per-
    // lane form).  The partner groups' partial sums are added at the end.
    constexpr int kQL = ROWS / SB;                // lanes per partner
    constexpr int kR = (NM + kQL - 1) / kQL;      // rows per lane
    static_assert(kQL * SB == ROWS && (kQL & (kQL - 1)) == 0, "partner groups");
    const int hq = (lane % ROWS) / kQL, rq = lane % kQL;
    const int i0 = kR * rq - PM;
    T accw[kR];
#pragma unroll
    for (int k = 0; k < kR; ++k) {
      accw[k].x = 0;
      accw[k].y = 0;
    }
    auto load_off = [&](int base) {
#pragma unroll
      for (int q = 0; q < PC; ++q) {
        const int e = lane + q * TH, s = e / (2 * NM);
        const bool ok = e < NCF && base + s < np;
        po[q] = ok ? nbr_off[pb0 + base + s] : -1;
        pp[q] = ok ? nbr_p[pb0 + base + s] : -1;
      }
    };
    auto load_val = [&](int base) {
      const int ns = min(SB, np - base);
      const double2 *src = nsym + ((int64_t)(pb0 + base) * 2) * NT;
#pragma unroll
      for (int q = 0; q < PS; ++q) {
        const int e = lane + q * TH;
        rs[q] = e < ns * 2 * NT ? sym_load(src + e) : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int q = 0; q < PC; ++q) {
        const int e = lane + q * TH;
        const int rem = e % (2 * NM), ww = rem / NM, jj = rem - ww * NM - PM;
        double2 v = make_double2(0.0, 0.0);
        if (po[q] >= 0 && jj >= -pp[q] && jj <= pp[q])
          v = xr[po[q] + ww * (2 * pp[q] + 1) + jj + pp[q]];
        rc[q] = v;
      }
    };
    load_off(0);
    load_val(0);
    load_off(SB);
    for (int base = 0; base < np; base += SB) {
#pragma unroll
      for (int q = 0; q < PS; ++q) {
        const int e = lane + q * TH;
        if (e < NSY) {
          const int s = e / (2 * NT), rem = e - s * 2 * NT;
          const int ww = rem / NT, kk = rem - ww * NT;
          t_lds[ww][s][kk] = CT<MIXED>::from(rs[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < PC; ++q) {
        const int e = lane + q * TH;
        if (e < NCF) {
          const int s = e / (2 * NM), rem = e - s * (2 * NM);
          const int ww = rem / NM, jj = rem - ww * NM;
          c_lds[s][ww][jj] = CT<MIXED>::from(rc[q]);
        }
      }
      __syncthreads();
      if (base + SB < np) {
        load_val(base + SB);
        load_off(base + 2 * SB);
      }
      {
        // entry of row i0 at coefficient jj: 3 PM + i0 - jj; rows past PM
        // (idle lanes) read clamped entries and are never stored
        const T *tw = t_lds[w][hq];
        const T *cw = c_lds[hq][w];
        T win[kR];
#pragma unroll
        for (int k = 1; k < kR; ++k) win[k] = tw[min(3 * PM + i0 + k, 4 * PM)];
#pragma unroll 4
        for (int jj = 0; jj < NM; ++jj) {
          win[0] = tw[min(3 * PM + i0 - jj, 4 * PM)];
          const T cv = cw[jj];
#pragma unroll
          for (int k = 0; k < kR; ++k) cfma_any(accw[k], win[k], cv);
#pragma unroll
          for (int k = kR - 1; k > 0; --k) win[k] = win[k - 1];
        }
      }
      __syncthreads();
    }
    // add the partner groups' partial sums (fixed order)
#pragma unroll
    for (int k = 0; k < kR; ++k) {
#pragma unroll
      for (int o = kQL; o < ROWS; o <<= 1) {
        accw[k].x += __shfl_xor(accw[k].x, o);
        accw[k].y += __shfl_xor(accw[k].y, o);
      }
    }
    if (hq == 0 && r0 < nrhs) {
#pragma unroll
      for (int k = 0; k < kR; ++k) {
        const int ir = i0 + k;
        if (ir >= -pb && ir <= pb)
          out[(int64_t)r0 * ldo + off[b] + w * (2 * pb + 1) + ir + pb] =
              make_double2((double)accw[k].x, (double)accw[k].y);
      }
    }
    return;
  }

  for (int base = 0; base < np; base += SB) {
    if (STORED) {
      // symbols of the near pairs, tabulated at set-up in near-list order
      const int ns = min(SB, np - base);
      const double2 *src = nsym + ((int64_t)(nbr_ptr[b] + base) * 2) * NT;
      for (int e = lane; e < SB * 2 * NT; e += 2 * ROWS) {
        const int s = e / (2 * NT), rem = e - s * 2 * NT;
        const int ww = rem / NT, kk = rem - ww * NT;
        t_lds[ww][s][kk] = CT<MIXED>::from(s < ns ? src[e] : make_double2(0.0, 0.0));
      }
    } else if (lane < 2 * SB) {
      const int s = lane >> 1, ww = lane & 1;
      const int l = base + s < np ? (nl ? nl[base + s] : base + s) : n;
      T *t = t_lds[ww][s];
      if (l < n && l != b) {
        // th_ml: angle of x_m - x_l (m target, l source of the forward map)
        double dx = bx - xy[2 * l], dy = by - xy[2 * l + 1];
        if (ADJ) {
          dx = -dx;
          dy = -dy;
        }
        graf_symbol<PM>(dx, dy, ww ? ks : kp, t, [](double2 v) { return CT<MIXED>::from(v); });
      } else {
        for (int k = 0; k < NT; ++k) {
          t[k].x = 0;
          t[k].y = 0;
        }
      }
    }
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      if (r0 + rr >= nrhs) break;  // uniform over the workgroup
      const double2 *xr = x + (int64_t)(r0 + rr) * ldx;
      for (int e = lane; e < SB * 2 * NM; e += 2 * ROWS) {
        const int s = e / (2 * NM), rem = e - s * (2 * NM);
        const int ww = rem / NM, jj = rem - ww * NM - PM;
        const int l = base + s < np ? (nl ? nl[base + s] : base + s) : n;
        double2 v = make_double2(0.0, 0.0);
        if (l < n && l != b) {
          const int pl = p[l];
          if (jj >= -pl && jj <= pl) v = xr[off[l] + ww * (2 * pl + 1) + jj + pl];
        }
        c_lds[s][ww][jj + PM] = CT<MIXED>::from(v);
      }
      __syncthreads();
      if (i <= PM) {
        for (int s = 0; s < SB; ++s) {
          // partial unroll: full unrolling hoists every LDS read into
          // registers and leaves one wavefront per SIMD
#pragma unroll 8
          for (int jj = 0; jj < NM; ++jj) {
            const int nu = i - (jj - PM);
            T tv = ADJ ? conj_any(t_lds[w][s][2 * PM - nu]) : t_lds[w][s][2 * PM + nu];
            cfma_any(acc[rr], tv, c_lds[s][w][jj]);
          }
        }
      }
      __syncthreads();
    }
  }
  if (i >= -pb && i <= pb) {
#pragma unroll
    for (int rr = 0; rr < RB; ++rr)
      if (r0 + rr < nrhs)
        out[(int64_t)(r0 + rr) * ldo + off[b] + w * (2 * pb + 1) + i + pb] =
            make_double2((double)acc[rr].x, (double)acc[rr].y);
  }
}

// Symbols of every near pair (forward orientation), for both wave numbers:
// nsym[(pair * 2 + w) * (4 PM + 1) + 2 PM + nu], pair = position in the near list.
template <int PM>
__global__ __launch_bounds__(256) void near_symbols_kernel(int npairs, const double *__restrict__ xy,
                                                           const int *__restrict__ pair_tgt,
                                                           const int *__restrict__ nbr_idx,
                                                           double kp, double ks,
                                                           double2 *__restrict__ nsym) {
  constexpr int NT = 4 * PM + 1;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 2 * (int64_t)npairs) return;
  const int pr = (int)(g >> 1), w = (int)(g & 1);
  const int b = pair_tgt[pr], l = nbr_idx[pr];
  graf_symbol<PM>(xy[2 * b] - xy[2 * l], xy[2 * b + 1] - xy[2 * l + 1], w ? ks : kp,
                  nsym + g * NT, [](double2 v) { return v; });
}

#define EMS_GRAF_LAUNCH(PMV, MIX, RBV, STV, ADV)                                             \
  hipLaunchKernelGGL((graf_direct_kernel<PMV, MIX, RBV, STV, ADV>),                             \
                     dim3(h->n, (nrhs + RBV - 1) / RBV), dim3(graf_threads(PMV)), 0, st, h->n,   \
                     nrhs, h->d_xy, h->d_p, h->d_off, x, h->ncoef, out, h->ncoef, h->md.kp,      \
                     h->md.ks, adjoint ? 1 : 0, nptr, nidx, h->d_nsym, h->d_nbr_off, h->d_nbr_p)
#define EMS_GRAF_RB(PMV, MIX, STV, ADV)                                                      \
  if (nrhs > 1) EMS_GRAF_LAUNCH(PMV, MIX, 8, STV, ADV);                                      \
  else EMS_GRAF_LAUNCH(PMV, MIX, 1, STV, ADV);
#define EMS_GRAF_GEN(PMV, MIX)                                                               \
  if (adjoint) { EMS_GRAF_RB(PMV, MIX, false, true) } else { EMS_GRAF_RB(PMV, MIX, false, false) }
#define EMS_GRAF_CASE(PMV)                                                                   \
  case PMV:                                                                                  \
    if (stored) {                                                                            \
      if (mixed) { EMS_GRAF_RB(PMV, true, true, false) } else { EMS_GRAF_RB(PMV, false, true, false) } \
    } else {                                                                                 \
      if (mixed) { EMS_GRAF_GEN(PMV, true) } else { EMS_GRAF_GEN(PMV, false) }                \
    }                                                                                        \
    break;

int pm_bucket(int pmax) {
  if (pmax <= 4) return 4;
  if (pmax <= 8) return 8;
  if (pmax <= 10) return 10;
  if (pmax <= 12) return 12;
  if (pmax <= 15) return 15;
  return 16;
}

static constexpr int graf_threads(int pm) { return 2 * pm + 1 <= 32 ? 64 : 128; }

hipError_t launch_graf_direct(const ems_handle *h, const double2 *x, double2 *out, int nrhs,
                              bool adjoint, bool mixed, hipStream_t st) {
  const int *nptr = h->fmm_on ? h->d_nbr_ptr : nullptr;
  const int *nidx = h->fmm_on ? h->d_nbr_idx : nullptr;
  // tabulated near-pair symbols serve the forward map (the adjoint with the
  // FMM runs the forward map through reciprocity)
  const bool stored = h->fmm_on && h->d_nsym != nullptr && !adjoint;
  switch (pm_bucket(h->pmax)) {
    EMS_GRAF_CASE(4)
    EMS_GRAF_CASE(8)
    EMS_GRAF_CASE(10)
    EMS_GRAF_CASE(12)
    EMS_GRAF_CASE(15)
    EMS_GRAF_CASE(16)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ems

namespace ems {

#define EMS_NSYM_CASE(PMV)                                                                   \
  case PMV:                                                                                  \
    hipLaunchKernelGGL((near_symbols_kernel<PMV>), dim3((unsigned)((2 * np + 255) / 256)),     \
                       dim3(256), 0, st, (int)np, h->d_xy, pair_tgt, h->d_nbr_idx, h->md.kp,   \
                       h->md.ks, h->d_nsym);                                                 \
    break;

hipError_t launch_near_symbols(ems_handle *h, const int *pair_tgt, hipStream_t st) {
  const int64_t np = h->n_pairs;
  if (np <= 0 || !h->d_nsym) return hipSuccess;
  switch (pm_bucket(h->pmax)) {
    EMS_NSYM_CASE(4)
    EMS_NSYM_CASE(8)
    EMS_NSYM_CASE(10)
    EMS_NSYM_CASE(12)
    EMS_NSYM_CASE(15)
    EMS_NSYM_CASE(16)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ems
