// Batched Toeplitz products for the free-space FMM: P2M, M2M, M2L (+L2L)
// and L2P are all out_k = sum_j s_{j-k} in_j with a tabulated symbol s (see
// fmm.cpp).  One workgroup owns one output expansion (or a 192-row chunk of
// it) and sweeps the tasks that feed it, so every output is written by exactly
// one workgroup (no atomics, fixed summation order).  The symbol window the
// chunk needs is staged in LDS; each lane forms R output coefficients from it
// and from the input vector read with scalar loads (see below).  Right-hand
// sides are taken 8 at a time, the symbol window of a task staged once for
// all of them.
#include "dev.h"
#include "ems_internal.h"

namespace ems {

// One wavefront per item; lane t owns the R consecutive output rows
// k_lo + R t + r.  For a fixed column j the symbols of those rows are
// s_{j-k}, consecutive entries of the staged window, so a lane keeps a ring
// of R of them and reads one new entry per column: one LDS read (stride R
// entries across lanes, conflict-free for odd R) per R complex multiply-adds.
// The input coefficient of column j is the same for every lane and is read
// with scalar loads straight from the expansion array.
// Launches whose outputs all have at most 64 rows (the particle-side L2P of
// orders up to 31) take R = 1, one row per lane: with R = 3 only a third of
// the lanes would hold rows.
constexpr int kToepR = 3;
constexpr int kToepRows = 64 * kToepR;
static_assert(kToepRows == kFmmRows, "item chunk of the plan");

template <int RB, int R>
__global__ __launch_bounds__(64) void toep_task_kernel(
    const int *__restrict__ ptr, const int64_t *__restrict__ in_base,
    const int *__restrict__ in_P, const int64_t *__restrict__ sym_base,
    const int *__restrict__ sym_L, const int *__restrict__ sgn,
    const int64_t *__restrict__ out_base, const int *__restrict__ out_P,
    const int *__restrict__ item_out, const int *__restrict__ item_row0,
    const int *__restrict__ item_t0, const int *__restrict__ item_t1,
    const int *__restrict__ item_slot, const double2 *__restrict__ in_main, int64_t in_stride,
    const double2 *__restrict__ in_alt, int64_t alt_stride, const double2 *__restrict__ pool,
    double2 *__restrict__ out, int64_t out_stride, double2 *__restrict__ part,
    int64_t part_stride, int accumulate, int max_in, int nrhs) {
  constexpr int ROWSR = 64 * R;            // rows of one item
  extern __shared__ double2 vs[];           // [2 max_in + kToepRows]
  const int item = blockIdx.x, r0 = blockIdx.y * RB, tid = threadIdx.x;
  const int o = item_out[item], row0 = item_row0[item];
  const int Po = out_P[o];
  const int rows = min(ROWSR, 2 * Po + 1 - row0);
  const int k_lo = -Po + row0, k_hi = k_lo + rows - 1;
  const int kb = k_lo + tid * R;            // first row of this lane
  const int b0 = k_hi - kb;                 // rows r <= b0 are inside the item
  double2 acc[RB][R];
#pragma unroll
  for (int rr = 0; rr < RB; ++rr)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[rr][r] = make_double2(0.0, 0.0);
  const int slot = item_slot[item];
  for (int t = item_t0[item]; t < item_t1[item]; ++t) {
    const int Pi = in_P[t], L = sym_L[t], sg = sgn[t];
    const int nin = 2 * Pi + 1;
    // window vs[e] = s_{nlo + e}, nlo = -Pi - k_hi (entry of column j, row k: j + Pi + k_hi - k)
    const int nlo = -Pi - k_hi;
    const int cnt = 2 * Pi + rows;
    const double2 *sym = pool + sym_base[t] + L;
    __syncthreads();
    for (int e = tid; e < cnt; e += 64) {
      const int nu = nlo + e;
      double2 v = sym[nu];
      if (sg == -1 && (nu & 1)) v = make_double2(-v.x, -v.y);
      vs[e] = v;
    }
    __syncthreads();
    if (b0 < 0) continue;                   // lane beyond the item's rows
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      if (r0 + rr >= nrhs) break;           // uniform over the wavefront
      const double2 *src =
          (sg == 2 ? in_alt + (int64_t)(r0 + rr) * alt_stride
                   : in_main + (int64_t)(r0 + rr) * in_stride) + in_base[t];
      // ring[m mod R] = window entry of (column m, row kb): vs[m + b0]
      double2 ring[R];
#pragma unroll
      for (int d = 1; d < R; ++d) ring[(R - d) % R] = vs[max(b0 - d, 0)];
      // two ring cycles per iteration (column index mod R stays compile-time)
      constexpr int U = 2 * R;
      int jj0 = 0;
      for (; jj0 + U <= nin; jj0 += U) {
#pragma unroll
        for (int d = 0; d < U; ++d) {
          ring[d % R] = vs[jj0 + d + b0];
          const double2 v = src[jj0 + d];
#pragma unroll
          for (int r = 0; r < R; ++r) cfma(acc[rr][r], ring[(d - r + U) % R], v);
        }
      }
#pragma unroll
      for (int d = 0; d < U; ++d) {
        if (jj0 + d < nin) {
          ring[d % R] = vs[jj0 + d + b0];
          const double2 v = src[jj0 + d];
#pragma unroll
          for (int r = 0; r < R; ++r) cfma(acc[rr][r], ring[(d - r + U) % R], v);
        }
      }
    }
  }
  if (b0 < 0) return;
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
    if (r0 + rr >= nrhs) break;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r > b0) break;                    // row beyond the item
      if (slot >= 0) {                      // partial over a group of the tasks
        part[(int64_t)(r0 + rr) * part_stride + (int64_t)slot * kFmmRows + (kb + r - k_lo)] =
            acc[rr][r];
        continue;
      }
      double2 *d = out + (int64_t)(r0 + rr) * out_stride + out_base[o] + (kb + r + Po);
      if (accumulate) *d = cadd(*d, acc[rr][r]);
      else *d = acc[rr][r];
    }
  }
}

// Sum of the task-group partials of one (output, chunk), in group order.
__global__ __launch_bounds__(kFmmRows) void fmm_reduce_kernel(
    const int *__restrict__ red_out, const int *__restrict__ red_row0,
    const int *__restrict__ red_slot0, const int *__restrict__ red_g,
    const int *__restrict__ out_P, const int64_t *__restrict__ out_base,
    const double2 *__restrict__ part, int64_t part_stride, double2 *__restrict__ out,
    int64_t out_stride, int accumulate) {
  const int k = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const int o = red_out[k], Po = out_P[o], row0 = red_row0[k];
  const int rows = min(kFmmRows, 2 * Po + 1 - row0);
  if (tid >= rows) return;
  const double2 *pp = part + (int64_t)r * part_stride + (int64_t)red_slot0[k] * kFmmRows + tid;
  double2 s = make_double2(0.0, 0.0);
  for (int g = 0; g < red_g[k]; ++g) s = cadd(s, pp[(int64_t)g * kFmmRows]);
  double2 *d = out + (int64_t)r * out_stride + out_base[o] + row0 + tid;
  if (accumulate) *d = cadd(*d, s);
  else *d = s;
}

hipError_t launch_fmm(const ems_handle *h, const double2 *x, double2 *fre, int nrhs,
                      hipStream_t st) {
  const FmmPlan &F = h->fmm;
  for (size_t li = 0; li < F.launches.size(); ++li) {
    const FmmLaunch &L = F.launches[li];
    const FmmDev &D = h->fmm_dev[li];
    const double2 *in = L.in_kind == 0 ? x : (L.in_kind == 1 ? h->d_mult : h->d_loc);
    const int64_t in_stride = L.in_kind == 0 ? h->ncoef : F.exp_len;
    double2 *out = L.out_kind == 1 ? h->d_mult : (L.out_kind == 2 ? h->d_loc : fre);
    const int64_t out_stride = L.out_kind == 3 ? h->ncoef : F.exp_len;
    const size_t lds = sizeof(double2) * (size_t)(2 * L.max_in_P + kToepRows);
    ProfScope ps(const_cast<ems_handle *>(h), L.name, st, L.flops * nrhs);
    const int64_t pst = (int64_t)F.max_slots * kFmmRows;
    const bool narrow = 2 * L.max_out_P + 1 <= 64;
#define EMS_TOEP_LAUNCH(RBV, RV)                                                               \
  hipLaunchKernelGGL((toep_task_kernel<RBV, RV>),                                              \
                     dim3((unsigned)L.item_out.size(), (nrhs + RBV - 1) / RBV), dim3(64), lds, st, \
                     D.ptr, D.in_base, D.in_P, D.sym_base, D.sym_L, D.sgn, D.out_base, D.out_P,   \
                     D.item_out, D.item_row0, D.item_t0, D.item_t1, D.item_slot, in, in_stride,   \
                     h->d_loc, F.exp_len, h->d_pool, out, out_stride, h->d_fmm_part, pst,        \
                     L.accumulate, L.max_in_P, nrhs)
    if (nrhs > 1) {
      if (narrow) EMS_TOEP_LAUNCH(8, 1);
      else EMS_TOEP_LAUNCH(8, kToepR);
    } else {
      if (narrow) EMS_TOEP_LAUNCH(1, 1);
      else EMS_TOEP_LAUNCH(1, kToepR);
    }
#undef EMS_TOEP_LAUNCH
    if (!L.red_out.empty())
      hipLaunchKernelGGL(fmm_reduce_kernel, dim3((unsigned)L.red_out.size(), nrhs), dim3(kFmmRows),
                         0, st, D.red_out, D.red_row0, D.red_slot0, D.red_g, D.out_P, D.out_base,
                         h->d_fmm_part, pst, out, out_stride, L.accumulate);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// v_m -> conj(P v_m) per particle block and wave, with (P v)_n = (-1)^n v_{-n}.
// The free-space operator is reciprocal, (T^{lm})^T = P T^{ml} P, so
// T^H v = P conj(T conj(P v)).
__global__ void conj_flip_kernel(const int *__restrict__ p, const int64_t *__restrict__ off,
                                 const double2 *__restrict__ in, double2 *__restrict__ out,
                                 int64_t ncoef) {
  const int m = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
  const int pm = p[m], N = 2 * pm + 1;
  if (lane >= 2 * N) return;
  const int w = lane < N ? 0 : 1;
  const int n = (w ? lane - N : lane) - pm;
  const int64_t b = (int64_t)r * ncoef + off[m] + w * N;
  double2 v = in[b + (-n) + pm];
  if (n & 1) v = make_double2(-v.x, -v.y);
  out[b + n + pm] = make_double2(v.x, -v.y);
}

hipError_t launch_conj_flip(const ems_handle *h, const double2 *in, double2 *out, int nrhs,
                            hipStream_t st) {
  hipLaunchKernelGGL(conj_flip_kernel, dim3(h->n, nrhs), dim3(part_threads(h)), 0, st, h->d_p, h->d_off, in, out,
                     h->ncoef);
  return hipGetLastError();
}

}  // namespace ems
