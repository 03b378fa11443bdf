// Right preconditioner of the GMRES solves: block Jacobi over spatial clusters
// of particles.  A cluster c collects a few neighbouring particles; its block
// of the free-space multiple-scattering system (Section 4.2, the
// S-preconditioned form: identity on the particle blocks, -S_m T^{ml} between
// particles m != l of the cluster, T^{ml} the Graf translation) is
//     B_c = I - S_c T_cc,
// inverted once per build and stored in complex64.  Applying the
// preconditioner maps every cluster's coefficients through B_c^{-1} (FP64
// arithmetic on the stored entries, so the preconditioner is one fixed linear
// map).  The reflected part and the couplings between clusters stay with
// GMRES; the preconditioner only has to absorb the strongest multiple
// scattering, which happens between close neighbours.
//
// Set-up per batch of clusters: the working matrices [B_c | I] (n2 rows,
// column-major, padded with identity rows and columns beyond the cluster's
// n_b unknowns) are filled, the off-diagonal particle blocks -S_m T^{ml} are
// assembled (one workgroup per ordered pair, symbols by the Graf recurrence),
// the batched LU with partial pivoting and the back substitution of the
// shapes generator turn the right half into B_c^{-1}, and its leading
// n_b x n_b block is packed column-major into the store.
#include "dev.h"
#include "ems_internal.h"
#include "graf_sym.h"

namespace ems {
namespace {

// [I | I] for every matrix of the batch (n2 x 2 n2, column-major).
__global__ __launch_bounds__(256) void pc_init_kernel(double2 *__restrict__ W, int n2,
                                                      int64_t mstride, int cnt) {
  const int64_t tot = (int64_t)n2 * 2 * n2;
  const int c = blockIdx.y;
  if (c >= cnt) return;
  double2 *A = W + (int64_t)c * mstride;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int col = (int)(e / n2), row = (int)(e % n2);
    const bool one = (col < n2 ? col : col - n2) == row;
    A[e] = make_double2(one ? 1.0 : 0.0, 0.0);
  }
}

// One workgroup per ordered pair (m, l), m != l, of a cluster: writes
// -(S_m T^{ml}) into the cluster's matrix at rows of m, columns of l.
// pairs[5 k .. 5 k + 4] = {matrix index in the batch, m, l, row offset of m,
// column offset of l inside the cluster}.
// (S_m T)[i][j] = sum_{k'} S_m[i][w N_m + k' + p_m] t^w_{k' - j'}, with j in
// wave w = j / N_l and j' = j % N_l - p_l (T is block diagonal in the waves).
__global__ __launch_bounds__(256) void pc_assemble_kernel(
    const int *__restrict__ pairs, int npairs, const double *__restrict__ xy,
    const int *__restrict__ p, const int64_t *__restrict__ Soff, const double2 *__restrict__ St,
    double kp, double ks, double2 *__restrict__ W, int n2, int64_t mstride) {
  constexpr int PM = kMaxP, NT = 4 * PM + 1;
  __shared__ double2 t[2][NT];
  const int k = blockIdx.x;
  if (k >= npairs) return;
  const int mat = pairs[5 * k], m = pairs[5 * k + 1], l = pairs[5 * k + 2];
  const int r0 = pairs[5 * k + 3], c0 = pairs[5 * k + 4];
  const int lane = threadIdx.x;
  if (lane < 2) {
    const double dx = xy[2 * m] - xy[2 * l], dy = xy[2 * m + 1] - xy[2 * l + 1];
    graf_symbol<PM>(dx, dy, lane ? ks : kp, t[lane], [](double2 v) { return v; });
  }
  __syncthreads();
  const int pm = p[m], pl = p[l];
  const int Nm = 2 * pm + 1, Nl = 2 * pl + 1, Km = 2 * Nm, Kl = 2 * Nl;
  const double2 *Sm = St + Soff[m];   // column-major: S_m[i][c] = Sm[c Km + i]
  double2 *A = W + (int64_t)mat * mstride;
  for (int e = lane; e < Km * Kl; e += 256) {
    const int i = e % Km, j = e / Km;
    const int w = j / Nl, jp = j % Nl - pl;
    double2 s = make_double2(0.0, 0.0);
    const double2 *tw = t[w] + 2 * PM - jp;
    for (int kk = 0; kk < Nm; ++kk) cfma(s, Sm[(int64_t)(w * Nm + kk) * Km + i], tw[kk - pm]);
    A[(int64_t)(c0 + j) * n2 + r0 + i] = make_double2(-s.x, -s.y);
  }
}

// inv[c] (n_b x n_b column-major, complex64) = the leading block of the right
// half of matrix c after the solve.
__global__ __launch_bounds__(256) void pc_pack_kernel(const double2 *__restrict__ W, int n2,
                                                      int64_t mstride, const int *__restrict__ nb,
                                                      const int64_t *__restrict__ ioff, int c0,
                                                      float2 *__restrict__ inv) {
  const int c = blockIdx.y;
  const int b = nb[c0 + c];
  const double2 *X = W + (int64_t)c * mstride + (int64_t)n2 * n2;
  float2 *o = inv + ioff[c0 + c];
  for (int e = blockIdx.x * 256 + threadIdx.x; e < b * b; e += gridDim.x * 256) {
    const int j = e / b, i = e % b;
    const double2 v = X[(int64_t)j * n2 + i];
    o[e] = make_float2((float)v.x, (float)v.y);
  }
}

// y = M^{-1} x on every cluster: one workgroup of kPcLanes lanes per
// (cluster, group of RB right-hand sides); the cluster's coefficients are
// gathered into LDS through rows[] (global coefficient index of each cluster
// row), lane i forms row i of B_c^{-1} x (column-major store: the lanes of a
// wave read one column coalesced) and scatters it back.  ADJ applies the
// conjugate transpose M^{-H} instead (lane i walks its own column: row i of
// (B_c^{-1})^H).
constexpr int kPcLanes = 512;
template <int RB, bool ADJ>
__global__ __launch_bounds__(kPcLanes) void pc_apply_kernel(
    const int *__restrict__ rptr, const int *__restrict__ rows, const int64_t *__restrict__ ioff,
    const float2 *__restrict__ inv, const double2 *__restrict__ x, double2 *__restrict__ y,
    int64_t ld, int nrhs) {
  __shared__ double2 xs[RB][kPcLanes];
  const int c = blockIdx.x, r0 = blockIdx.y * RB;
  const int b = rptr[c + 1] - rptr[c];
  const int *rw = rows + rptr[c];
  const int i = threadIdx.x;
  int gi = 0;
  if (i < b) {
    gi = rw[i];
#pragma unroll
    for (int q = 0; q < RB; ++q)
      xs[q][i] = r0 + q < nrhs ? x[(int64_t)(r0 + q) * ld + gi] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (i >= b) return;
  // entry (i, j) of the applied block at Ic[j * js]: column-major B_c^{-1},
  // or its transpose (conjugated) for the adjoint
  const float2 *Ic = inv + ioff[c] + (ADJ ? (int64_t)i * b : i);
  const int64_t js = ADJ ? 1 : b;
  const double cs = ADJ ? -1.0 : 1.0;
  double2 acc[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q) acc[q] = make_double2(0.0, 0.0);
  int j = 0;
  for (; j + 4 <= b; j += 4) {
    float2 e[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) e[u] = Ic[(int64_t)(j + u) * js];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double2 ed = make_double2((double)e[u].x, cs * (double)e[u].y);
#pragma unroll
      for (int q = 0; q < RB; ++q) cfma(acc[q], ed, xs[q][j + u]);
    }
  }
  for (; j < b; ++j) {
    const float2 e = Ic[(int64_t)j * js];
    const double2 ed = make_double2((double)e.x, cs * (double)e.y);
#pragma unroll
    for (int q = 0; q < RB; ++q) cfma(acc[q], ed, xs[q][j]);
  }
#pragma unroll
  for (int q = 0; q < RB; ++q)
    if (r0 + q < nrhs) y[(int64_t)(r0 + q) * ld + gi] = acc[q];
}

}  // namespace

hipError_t launch_pc_factor_batch(const ems_handle *h, const PcBatch &bt, double2 *W, int n2,
                                  int64_t mstride, int *info, hipStream_t st) {
  if (n2 > kPcLanes || bt.cnt <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pc_init_kernel, dim3(64, bt.cnt), dim3(256), 0, st, W, n2, mstride, bt.cnt);
  if (bt.npairs > 0)
    hipLaunchKernelGGL(pc_assemble_kernel, dim3(bt.npairs), dim3(256), 0, st, bt.pairs,
                       bt.npairs, h->d_xy, h->d_p, h->d_Soff, h->d_S, h->md.kp, h->md.ks, W, n2,
                       mstride);
  hipError_t e = launch_lu_solve_batch(W, n2, mstride, bt.cnt, n2, info, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pc_pack_kernel, dim3(64, bt.cnt), dim3(256), 0, st, W, n2, mstride,
                     h->d_pc_nb, h->d_pc_ioff, bt.c0, h->d_pc_inv);
  return hipGetLastError();
}

hipError_t launch_pc_apply(const ems_handle *h, const double2 *x, double2 *y, int nrhs,
                           bool adjoint, hipStream_t st) {
  const int64_t ld = h->ncoef;
#define EMS_PC_LAUNCH(RB, ADJ)                                                              \
  hipLaunchKernelGGL((pc_apply_kernel<RB, ADJ>), dim3(h->pc_nc, (nrhs + RB - 1) / RB),      \
                     dim3(kPcLanes), 0, st, h->d_pc_rptr, h->d_pc_rows, h->d_pc_ioff,        \
                     h->d_pc_inv, x, y, ld, nrhs)
  if (nrhs >= 4) {
    if (adjoint) EMS_PC_LAUNCH(4, true);
    else EMS_PC_LAUNCH(4, false);
  } else {
    if (adjoint) EMS_PC_LAUNCH(1, true);
    else EMS_PC_LAUNCH(1, false);
  }
#undef EMS_PC_LAUNCH
  return hipGetLastError();
}

}  // namespace ems
