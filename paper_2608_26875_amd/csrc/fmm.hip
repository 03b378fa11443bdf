// Batched Toeplitz products for the free-space FMM: P2M, M2M, M2L (+L2L)
// and L2P are all out_k = sum_j s_{j-k} in_j with a tabulated symbol s (see
// fmm.cpp).  One workgroup owns one output expansion (or a 256-row chunk of
// it) and sweeps the tasks that feed it, so every output is written by exactly
// one workgroup (no atomics, fixed summation order).  The input vector and
// the symbol window the chunk needs are staged in LDS; each lane then forms
// one output coefficient.  Right-hand sides are taken 8 at a time, the
// symbol window of a task staged once for all of them.
#include "dev.h"
#include "ems_internal.h"

namespace ems {

template <int RB>
__global__ __launch_bounds__(256) void toep_task_kernel(
    const int *__restrict__ ptr, const int64_t *__restrict__ in_base,
    const int *__restrict__ in_P, const int64_t *__restrict__ sym_base,
    const int *__restrict__ sym_L, const int *__restrict__ sgn,
    const int64_t *__restrict__ out_base, const int *__restrict__ out_P,
    const int *__restrict__ item_out, const int *__restrict__ item_row0,
    const double2 *__restrict__ in_main, int64_t in_stride, const double2 *__restrict__ in_alt,
    int64_t alt_stride, const double2 *__restrict__ pool, double2 *__restrict__ out,
    int64_t out_stride, int accumulate, int max_in, int nrhs) {
  extern __shared__ double2 lds[];
  double2 *vin = lds;                       // [2 max_in + 1]
  double2 *vs = lds + 2 * max_in + 1;       // [2 max_in + 256]
  const int item = blockIdx.x, r0 = blockIdx.y * RB, tid = threadIdx.x;
  const int o = item_out[item], row0 = item_row0[item];
  const int Po = out_P[o];
  const int rows = min(256, 2 * Po + 1 - row0);
  const int k_lo = -Po + row0, k_hi = k_lo + rows - 1;
  const int k = k_lo + tid;
  double2 acc[RB];
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) acc[rr] = make_double2(0.0, 0.0);
  for (int t = ptr[o]; t < ptr[o + 1]; ++t) {
    const int Pi = in_P[t], L = sym_L[t], sg = sgn[t];
    const int nin = 2 * Pi + 1;
    // the symbol window of this task serves every right-hand side of the chunk
    const int nlo = -Pi - k_hi;
    const int cnt = 2 * Pi + rows;
    const double2 *sym = pool + sym_base[t] + L;
    for (int e = tid; e < cnt; e += 256) {
      const int nu = nlo + e;
      double2 v = sym[nu];
      if (sg == -1 && (nu & 1)) v = make_double2(-v.x, -v.y);
      vs[e] = v;
    }
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      const int r = r0 + rr;
      if (r >= nrhs) break;  // uniform over the workgroup
      const double2 *src =
          (sg == 2 ? in_alt + (int64_t)r * alt_stride : in_main + (int64_t)r * in_stride) + in_base[t];
      for (int e = tid; e < nin; e += 256) vin[e] = src[e];
      __syncthreads();
      if (tid < rows) {
        // nu = j - k, index (j + Pi) + (k_hi - k)
        const double2 *s0 = vs + (k_hi - k);
        for (int jj = 0; jj < nin; ++jj) cfma(acc[rr], s0[jj], vin[jj]);
      }
      __syncthreads();
    }
  }
  if (tid < rows) {
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      if (r0 + rr >= nrhs) break;
      double2 *d = out + (int64_t)(r0 + rr) * out_stride + out_base[o] + (k + Po);
      if (accumulate) *d = cadd(*d, acc[rr]);
      else *d = acc[rr];
    }
  }
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
    const size_t lds = sizeof(double2) * (size_t)(4 * L.max_in_P + 257);
    ProfScope ps(const_cast<ems_handle *>(h), L.name, st, L.flops * nrhs);
    if (nrhs > 1)
      hipLaunchKernelGGL((toep_task_kernel<8>), dim3((unsigned)L.item_out.size(), (nrhs + 7) / 8),
                         dim3(256), lds, st, D.ptr, D.in_base, D.in_P, D.sym_base, D.sym_L, D.sgn,
                         D.out_base, D.out_P, D.item_out, D.item_row0, in, in_stride, h->d_loc,
                         F.exp_len, h->d_pool, out, out_stride, L.accumulate, L.max_in_P, nrhs);
    else
      hipLaunchKernelGGL((toep_task_kernel<1>), dim3((unsigned)L.item_out.size(), 1), dim3(256),
                         lds, st, D.ptr, D.in_base, D.in_P, D.sym_base, D.sym_L, D.sgn, D.out_base,
                         D.out_P, D.item_out, D.item_row0, in, in_stride, h->d_loc, F.exp_len,
                         h->d_pool, out, out_stride, L.accumulate, L.max_in_P, nrhs);
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
