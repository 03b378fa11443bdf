// Layered reflected part of the operator on a Sommerfeld node set (Section 4).
//
//   aggregate   (multipole-to-Sommerfeld, Section 4.4 Lemma):
//       I_w(j) = sum_m e^{s_w(j) y_m - i xi_j x_m} sum_n c^m_{w,n} (-i zeta_w(j))^n
//   reflect     (interface, Section 2.2 per node; Schur complement, Section 4.2):
//       [RP; RS]_j = w_j R(xi_j) [I_p / (i pi s_p); I_s / (i pi s_s)]
//   disaggregate (Sommerfeld-to-local, Section 4.3, Jacobi-Anger):
//       a^l_{w,n} = sum_j e^{i xi_j x_l + s_w(j) y_l} (i zeta_w(j))^n RW_j
// with w in {P, S}, zeta = (xi - s)/k, and (i zeta)^n = (-1)^n (-i zeta)^n so a
// single power table V[j][n] = (-i zeta_w(j))^n serves both contractions (the
// (-1)^n is applied when the partial sums are combined).
//
// The adjoint (conjugate transpose) runs the same two kernels with the roles
// swapped: the aggregate kernel evaluates D^H (conjugated disaggregate
// factors), the reflect kernel applies conj(w) R^H conj(1/(i pi s)), the
// disaggregate kernel evaluates A^H.
//
// Layout: lanes own nodes (aggregate) or particles (disaggregate); the other
// index is swept in a wave-uniform loop, so the coefficient or power-table
// operand is the same for every lane.  Per (node, particle) pair one complex
// exponential is formed in FP64 and (2p+1) complex multiply-adds follow.
// Partial sums over particle chunks (aggregate) and node chunks
// (disaggregate) are written separately and reduced in a fixed order, so
// results are reproducible run to run.
#include "dev.h"
#include "ems_internal.h"

namespace ems {

int pm_bucket(int pmax);

// MODE 0: forward with tabulated exponentials, 1: forward, exponentials
// formed on the fly, 2: adjoint (on the fly).
template <int PM, bool UNI, int MODE>
__global__ __launch_bounds__(256) void somm_aggregate_kernel(
    int n, int q, int pmax, const double *__restrict__ xy, const int *__restrict__ p,
    const int64_t *__restrict__ off, const double2 *__restrict__ x, int64_t ldx,
    const double2 *__restrict__ xi_t, const double2 *__restrict__ sp_t,
    const double2 *__restrict__ ss_t, const double2 *__restrict__ Vp_t,
    const double2 *__restrict__ Vs_t, double2 *__restrict__ agg, int chunks, int per_chunk,
    int adjoint_unused, const double2 *__restrict__ Etab) {
  constexpr int NM = 2 * PM + 1;
  constexpr bool TAB = MODE == 0;
  constexpr bool adjoint = MODE == 2;
  (void)adjoint_unused;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  const int wave = blockIdx.z & 1;
  const int r = blockIdx.z >> 1;
  const int jj = j < q ? j : q - 1;
  const double2 *Vt = wave ? Vs_t : Vp_t;
  const double2 xi = xi_t[jj];
  const double2 s = wave ? ss_t[jj] : sp_t[jj];
  // power tables are padded to the kernel order PM (zeros beyond pmax)
  const int ld = 2 * PM + 1;
  (void)pmax;
  // exponent a y + b x
  double2 a, bb;
  if (!adjoint) {
    a = s;
    bb = make_double2(xi.y, -xi.x);   // -i xi
  } else {
    a = cconj(s);
    bb = make_double2(-xi.y, -xi.x);  // conj(i xi)
  }
  double2 v[NM];
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    const int nn = k - PM;
    double2 t = Vt[(int64_t)jj * ld + k];
    if (adjoint) {
      t = cconj(t);
      if (nn & 1) t = cscale(t, -1.0);
    }
    v[k] = t;
  }
  // acc_n = sum_m E(j, m) c^m_n, then I = sum_n V[j][n] acc_n: the 2p+1
  // accumulators are independent chains (same flop count as contracting the
  // modes first).
  double2 acc[NM];
#pragma unroll
  for (int k = 0; k < NM; ++k) acc[k] = make_double2(0.0, 0.0);
  const int m0 = c * per_chunk;
  const int m1 = min(n, m0 + per_chunk);
  const double2 *xr = x + (int64_t)r * ldx;
  // tabulated exponentials E[wave][m][j] (forward only)
  const double2 *Ew = TAB ? Etab + (int64_t)wave * n * q + jj : nullptr;
  for (int m = m0; m < m1; ++m) {
    const int pm = UNI ? PM : p[m];
    const double2 *cm = xr + (UNI ? (int64_t)m * 2 * (2 * PM + 1) : off[m]) + wave * (2 * pm + 1) + pm;
    double2 E;
    if (TAB) {
      E = Ew[(int64_t)m * q];
    } else {
      const double xm = xy[2 * m], ym = xy[2 * m + 1];
      E = cexp(make_double2(a.x * ym + bb.x * xm, a.y * ym + bb.y * xm));
    }
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      const int nn = k - PM;
      if (UNI || (nn >= -pm && nn <= pm)) cfma(acc[k], E, cm[nn]);
    }
  }
  double2 res = make_double2(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < NM; ++k) cfma(res, v[k], acc[k]);
  if (j < q) agg[((int64_t)(r * 2 + wave) * chunks + c) * q + j] = res;
}

__global__ void somm_reflect_kernel(int q, int chunks, const double2 *__restrict__ agg,
                                    const double2 *__restrict__ w_t,
                                    const double2 *__restrict__ sp_t,
                                    const double2 *__restrict__ ss_t,
                                    const double2 *__restrict__ R_t, double2 *__restrict__ g,
                                    int adjoint) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (j >= q) return;
  double2 Ip = make_double2(0.0, 0.0), Is = make_double2(0.0, 0.0);
  for (int c = 0; c < chunks; ++c) {
    Ip = cadd(Ip, agg[((int64_t)(r * 2 + 0) * chunks + c) * q + j]);
    Is = cadd(Is, agg[((int64_t)(r * 2 + 1) * chunks + c) * q + j]);
  }
  const double kInvPi = 0.31830988618379067154;
  // 1 / (i pi s) = -i / (pi s)
  const double2 sp = sp_t[j], ss = ss_t[j];
  const double dp = sp.x * sp.x + sp.y * sp.y, ds = ss.x * ss.x + ss.y * ss.y;
  const double2 cp = make_double2(-sp.y * kInvPi / dp, -sp.x * kInvPi / dp);
  const double2 cs = make_double2(-ss.y * kInvPi / ds, -ss.x * kInvPi / ds);
  const double2 *R = R_t + 4 * (int64_t)j;
  const double2 w = w_t[j];
  double2 op, os;
  if (!adjoint) {
    const double2 up = cmul(Ip, cp), us = cmul(Is, cs);
    op = cmul(w, cadd(cmul(R[0], up), cmul(R[1], us)));
    os = cmul(w, cadd(cmul(R[2], up), cmul(R[3], us)));
  } else {
    const double2 tp = cmul(cconj(w), Ip), ts = cmul(cconj(w), Is);
    const double2 up = cadd(cmul(cconj(R[0]), tp), cmul(cconj(R[2]), ts));
    const double2 us = cadd(cmul(cconj(R[1]), tp), cmul(cconj(R[3]), ts));
    op = cmul(cconj(cp), up);
    os = cmul(cconj(cs), us);
  }
  g[(int64_t)(r * 2 + 0) * q + j] = op;
  g[(int64_t)(r * 2 + 1) * q + j] = os;
}

template <int PM, int MODE>
__global__ __launch_bounds__(256) void somm_disaggregate_kernel(
    int n, int q, int pmax, const double *__restrict__ xy, const int *__restrict__ p,
    const int64_t *__restrict__ off, const double2 *__restrict__ xi_t,
    const double2 *__restrict__ sp_t, const double2 *__restrict__ ss_t,
    const double2 *__restrict__ Vp_t, const double2 *__restrict__ Vs_t,
    const double2 *__restrict__ g, double2 *__restrict__ dis, int64_t ncoef, int chunks,
    int per_chunk, int adjoint_unused, const double2 *__restrict__ Etab) {
  constexpr int NM = 2 * PM + 1;
  constexpr bool TAB = MODE == 0;
  constexpr bool adjoint = MODE == 2;
  (void)adjoint_unused;
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  const int wave = blockIdx.z & 1;
  const int r = blockIdx.z >> 1;
  const int ll = l < n ? l : n - 1;
  const double xl = xy[2 * ll], yl = xy[2 * ll + 1];
  const int pl = p[ll];
  const int ld = 2 * PM + 1;
  (void)pmax;
  const double2 *Vt = wave ? Vs_t : Vp_t;
  const double2 *st = wave ? ss_t : sp_t;
  const double2 *gr = g + (int64_t)(r * 2 + wave) * q;
  double2 acc[NM];
#pragma unroll
  for (int k = 0; k < NM; ++k) acc[k] = make_double2(0.0, 0.0);
  const int j0 = c * per_chunk;
  const int j1 = min(q, j0 + per_chunk);
  // tabulated exponentials E[wave][j][l] (forward only)
  const double2 *Ew = TAB ? Etab + (int64_t)wave * q * n + ll : nullptr;
  for (int j = j0; j < j1; ++j) {
    double2 E;
    if (TAB) {
      E = Ew[(int64_t)j * n];
    } else {
      const double2 xi = xi_t[j];
      const double2 s = st[j];
      double2 a, bb;
      if (!adjoint) {
        a = s;
        bb = make_double2(-xi.y, xi.x);  // i xi
      } else {
        a = cconj(s);
        bb = make_double2(xi.y, xi.x);   // conj(-i xi)
      }
      E = cexp(make_double2(a.x * yl + bb.x * xl, a.y * yl + bb.y * xl));
    }
    const double2 F = cmul(E, gr[j]);
    const double2 *Vj = Vt + (int64_t)j * ld;
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      double2 u = Vj[k];
      if (adjoint) u = cconj(u);
      cfma(acc[k], F, u);
    }
  }
  if (l < n) {
    double2 *o = dis + ((int64_t)r * chunks + c) * ncoef + off[l] + wave * (2 * pl + 1) + pl;
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      const int nn = k - PM;
      if (nn >= -pl && nn <= pl) o[nn] = acc[k];
    }
  }
}

#define EMS_AGG_LAUNCH(PMV, UNIV, TABV)                                                    \
  hipLaunchKernelGGL((somm_aggregate_kernel<PMV, UNIV, TABV>), grid, dim3(256), 0, st, h->n,  \
                     h->q, h->pmax, h->d_xy, h->d_p, h->d_off, x, h->ncoef, h->d_xi, h->d_sp,  \
                     h->d_ss, h->d_Vp, h->d_Vs, h->d_agg, h->agg_chunks, per, adjoint ? 1 : 0,  \
                     h->d_Eagg)
#define EMS_AGG_CASE(PMV)                                                                  \
  case PMV:                                                                                \
    if (mode == 0 && uni) EMS_AGG_LAUNCH(PMV, true, 0);                                    \
    else if (mode == 0) EMS_AGG_LAUNCH(PMV, false, 0);                                     \
    else if (mode == 1 && uni) EMS_AGG_LAUNCH(PMV, true, 1);                               \
    else if (mode == 1) EMS_AGG_LAUNCH(PMV, false, 1);                                     \
    else EMS_AGG_LAUNCH(PMV, false, 2);                                                    \
    break;

hipError_t launch_somm_aggregate(const ems_handle *h, const double2 *x, int nrhs, bool adjoint,
                                 bool mixed, hipStream_t st) {
  (void)mixed;
  const int per = (h->n + h->agg_chunks - 1) / h->agg_chunks;
  dim3 grid((h->q + 255) / 256, h->agg_chunks, 2 * nrhs);
  const int pb = pm_bucket(h->pmax);
  const int mode = adjoint ? 2 : (h->d_Eagg != nullptr ? 0 : 1);
  const bool uni = h->p_uniform && pb == h->pmax;
  switch (pb) {
    EMS_AGG_CASE(4)
    EMS_AGG_CASE(8)
    EMS_AGG_CASE(10)
    EMS_AGG_CASE(12)
    EMS_AGG_CASE(15)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_somm_reflect(const ems_handle *h, int nrhs, bool adjoint, hipStream_t st) {
  dim3 grid((h->q + 255) / 256, nrhs);
  hipLaunchKernelGGL(somm_reflect_kernel, grid, dim3(256), 0, st, h->q, h->agg_chunks, h->d_agg,
                     h->d_w, h->d_sp, h->d_ss, h->d_R, h->d_refl, adjoint ? 1 : 0);
  return hipGetLastError();
}

#define EMS_DIS_LAUNCH(PMV, TABV)                                                          \
  hipLaunchKernelGGL((somm_disaggregate_kernel<PMV, TABV>), grid, dim3(256), 0, st, h->n, h->q, \
                     h->pmax, h->d_xy, h->d_p, h->d_off, h->d_xi, h->d_sp, h->d_ss, h->d_Vp,    \
                     h->d_Vs, h->d_refl, h->d_dis, h->ncoef, h->dis_chunks, per,               \
                     adjoint ? 1 : 0, h->d_Edis)
#define EMS_DIS_CASE(PMV)                                                                  \
  case PMV:                                                                                \
    if (mode == 0) EMS_DIS_LAUNCH(PMV, 0);                                                 \
    else if (mode == 1) EMS_DIS_LAUNCH(PMV, 1);                                            \
    else EMS_DIS_LAUNCH(PMV, 2);                                                           \
    break;

hipError_t launch_somm_disaggregate(const ems_handle *h, int nrhs, bool adjoint, bool mixed,
                                    hipStream_t st) {
  (void)mixed;
  const int per = (h->q + h->dis_chunks - 1) / h->dis_chunks;
  dim3 grid((h->n + 255) / 256, h->dis_chunks, 2 * nrhs);
  const int mode = adjoint ? 2 : (h->d_Edis != nullptr ? 0 : 1);
  switch (pm_bucket(h->pmax)) {
    EMS_DIS_CASE(4)
    EMS_DIS_CASE(8)
    EMS_DIS_CASE(10)
    EMS_DIS_CASE(12)
    EMS_DIS_CASE(15)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Tables of the geometry-dependent exponentials (set-up, once per geometry
// and frequency):  Eagg[w][m][j] = e^{s_w(j) y_m - i xi_j x_m},
// Edis[w][j][l] = e^{i xi_j x_l + s_w(j) y_l}.
__global__ void etab_agg_kernel(int n, int q, const double *__restrict__ xy,
                                const double2 *__restrict__ xi_t, const double2 *__restrict__ sp_t,
                                const double2 *__restrict__ ss_t, double2 *__restrict__ E) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  const int w = blockIdx.z;
  if (j >= q) return;
  const double2 xi = xi_t[j];
  const double2 s = w ? ss_t[j] : sp_t[j];
  const double xm = xy[2 * m], ym = xy[2 * m + 1];
  // s y - i xi x
  E[((int64_t)w * n + m) * q + j] = cexp(make_double2(s.x * ym + xi.y * xm, s.y * ym - xi.x * xm));
}

__global__ void etab_dis_kernel(int n, int q, const double *__restrict__ xy,
                                const double2 *__restrict__ xi_t, const double2 *__restrict__ sp_t,
                                const double2 *__restrict__ ss_t, double2 *__restrict__ E) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int w = blockIdx.z;
  if (l >= n) return;
  const double2 xi = xi_t[j];
  const double2 s = w ? ss_t[j] : sp_t[j];
  const double xl = xy[2 * l], yl = xy[2 * l + 1];
  // i xi x + s y
  E[((int64_t)w * q + j) * n + l] = cexp(make_double2(s.x * yl - xi.y * xl, s.y * yl + xi.x * xl));
}

hipError_t launch_etables(ems_handle *h, hipStream_t st) {
  hipLaunchKernelGGL(etab_agg_kernel, dim3((h->q + 255) / 256, h->n, 2), dim3(256), 0, st, h->n,
                     h->q, h->d_xy, h->d_xi, h->d_sp, h->d_ss, h->d_Eagg);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(etab_dis_kernel, dim3((h->n + 255) / 256, h->q, 2), dim3(256), 0, st, h->n,
                     h->q, h->d_xy, h->d_xi, h->d_sp, h->d_ss, h->d_Edis);
  return hipGetLastError();
}

}  // namespace ems
