// Scattered displacement at host points (y < 0; Section 5, coupled
// representation; substrate points y > 0 see the transmitted part only):
//   u(x) = sum_m sum_n alpha^m_n grad v_n^{kp}(x - x_m) + beta^m_n grad^perp v_n^{ks}(x - x_m)
//          + grad phi_R + grad^perp psi_R,
// v_n^k = H_n(k r) e^{i n theta}, d_x v_n = (k/2)(v_{n-1} - v_{n+1}),
// d_y v_n = (i k/2)(v_{n-1} + v_{n+1}); phi_R = sum_j e^{i xi_j x + s_p y} RP_j and
// psi_R likewise with RS (the reflected amplitudes of the aggregate/reflect
// stages, quadrature weights included), so grad -> (i xi, s_p) and
// grad^perp -> (-s_s, i xi).
#include "dev.h"
#include "ems_internal.h"

namespace ems {

// lane = receiver point; every particle is visited (direct sum).
template <int PM>
__global__ __launch_bounds__(256) void field_direct_kernel(
    int n, int npts, const double *__restrict__ xy, const int *__restrict__ p,
    const int64_t *__restrict__ off, const double2 *__restrict__ gam, int64_t ldg,
    const double *__restrict__ pts, double2 *__restrict__ u, double kp, double ks) {
  constexpr int L = PM + 1;  // orders -L..L of v_k are needed
  const int ip = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  const int ipc = ip < npts ? ip : npts - 1;
  const double px = pts[2 * ipc], py = pts[2 * ipc + 1];
  const double2 *g = gam + (int64_t)r * ldg;
  double2 ux = make_double2(0.0, 0.0), uy = make_double2(0.0, 0.0);
  // receivers in the substrate (y > 0) see only the transmitted field
  const int nm = py < 0.0 ? n : 0;
  for (int m = 0; m < nm; ++m) {
    const double dx = px - xy[2 * m], dy = py - xy[2 * m + 1];
    const double rr = sqrt(dx * dx + dy * dy);
    const double th = atan2(dy, dx);
    double sn, cs;
    sincos(th, &sn, &cs);
    const double2 e1 = make_double2(cs, sn);  // e^{i theta}
    const int pm = p[m];
    const double2 *al = g + off[m] + pm;            // alpha_n at al[n]
    const double2 *be = g + off[m] + 2 * pm + 1 + pm;  // beta_n at be[n]
    for (int w = 0; w < 2; ++w) {
      const double k = w ? ks : kp;
      const double z = k * rr;
      // v_k for k = 0..L: H_k e^{i k theta}; v_{-k} = (-1)^k H_k e^{-i k theta}
      double2 vp[L + 1], vn[L + 1];
      double2 hm = make_double2(j0(z), y0(z)), h = make_double2(j1(z), y1(z));
      vp[0] = hm;
      vn[0] = hm;
      double2 ph = e1;
      vp[1] = cmul(h, ph);
      vn[1] = cscale(cmul(h, cconj(ph)), -1.0);
      const double iz = 2.0 / z;
#pragma unroll
      for (int kk = 2; kk <= L; ++kk) {
        const double2 hn = csub(cscale(h, (kk - 1) * iz), hm);
        hm = h;
        h = hn;
        ph = cmul(ph, e1);
        vp[kk] = cmul(h, ph);
        vn[kk] = cscale(cmul(h, cconj(ph)), (kk & 1) ? -1.0 : 1.0);
      }
      // sum_n c_n (v_{n-1} -+ v_{n+1})
      double2 dif = make_double2(0.0, 0.0), sum = make_double2(0.0, 0.0);
      const double2 *c = w ? be : al;
#pragma unroll
      for (int nn = -PM; nn <= PM; ++nn) {
        if (nn < -pm || nn > pm) continue;
        const int a1 = nn - 1, a2 = nn + 1;
        const double2 v1 = a1 >= 0 ? vp[a1] : vn[-a1];
        const double2 v2 = a2 >= 0 ? vp[a2] : vn[-a2];
        const double2 cn = c[nn];
        cfma(dif, cn, csub(v1, v2));
        cfma(sum, cn, cadd(v1, v2));
      }
      // d_x part (k/2) dif, d_y part (i k/2) sum
      const double2 gx = cscale(dif, 0.5 * k);
      const double2 gy = make_double2(-0.5 * k * sum.y, 0.5 * k * sum.x);
      if (w == 0) {
        ux = cadd(ux, gx);
        uy = cadd(uy, gy);
      } else {  // grad^perp = (-d_y, d_x)
        ux = csub(ux, gy);
        uy = cadd(uy, gx);
      }
    }
  }
  if (ip < npts) {
    double2 *o = u + ((int64_t)r * npts + ip) * 2;
    o[0] = ux;
    o[1] = uy;
  }
}

// lane = receiver; sum over the Sommerfeld nodes of the reflected potentials.
__global__ __launch_bounds__(256) void field_refl_kernel(
    int q, int npts, const double2 *__restrict__ xi_t, const double2 *__restrict__ sp_t,
    const double2 *__restrict__ ss_t, const double2 *__restrict__ g, const double *__restrict__ pts,
    double2 *__restrict__ u) {
  const int ip = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (ip >= npts) return;
  const double px = pts[2 * ip], py = pts[2 * ip + 1];
  if (!(py < 0.0)) return;  // host receivers only
  const double2 *RP = g + (int64_t)(r * 2 + 0) * q;
  const double2 *RS = g + (int64_t)(r * 2 + 1) * q;
  double2 ux = make_double2(0.0, 0.0), uy = make_double2(0.0, 0.0);
  for (int j = 0; j < q; ++j) {
    const double2 xi = xi_t[j], sp = sp_t[j], ss = ss_t[j];
    const double2 ixi = make_double2(-xi.y, xi.x);
    // e^{i xi x + s y}
    const double2 ep = cmul(cexp(make_double2(-xi.y * px + sp.x * py, xi.x * px + sp.y * py)), RP[j]);
    const double2 es = cmul(cexp(make_double2(-xi.y * px + ss.x * py, xi.x * px + ss.y * py)), RS[j]);
    ux = cadd(ux, csub(cmul(ixi, ep), cmul(ss, es)));
    uy = cadd(uy, cadd(cmul(sp, ep), cmul(ixi, es)));
  }
  double2 *o = u + ((int64_t)r * npts + ip) * 2;
  o[0] = cadd(o[0], ux);
  o[1] = cadd(o[1], uy);
}


// Transmitted part at substrate receivers (y > 0): the particles' upgoing
// potentials cross the interface as e^{i xi x - s_b y} TP_j (P) and TS_j (S),
// the substrate's upgoing potentials (weights included); grad -> (i xi,
// -s_pb), grad^perp -> (s_sb, i xi).
__global__ __launch_bounds__(256) void field_trans_kernel(
    int q, int npts, const double2 *__restrict__ xi_t, const double2 *__restrict__ spb_t,
    const double2 *__restrict__ ssb_t, const double2 *__restrict__ g,
    const double *__restrict__ pts, double2 *__restrict__ u) {
  const int ip = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (ip >= npts) return;
  const double px = pts[2 * ip], py = pts[2 * ip + 1];
  if (!(py > 0.0)) return;
  const double2 *TP = g + (int64_t)(r * 2 + 0) * q;
  const double2 *TS = g + (int64_t)(r * 2 + 1) * q;
  double2 ux = make_double2(0.0, 0.0), uy = make_double2(0.0, 0.0);
  for (int j = 0; j < q; ++j) {
    const double2 xi = xi_t[j], sp = spb_t[j], ss = ssb_t[j];
    const double2 ixi = make_double2(-xi.y, xi.x);
    // e^{i xi x - s y}
    const double2 ep = cmul(cexp(make_double2(-xi.y * px - sp.x * py, xi.x * px - sp.y * py)), TP[j]);
    const double2 es = cmul(cexp(make_double2(-xi.y * px - ss.x * py, xi.x * px - ss.y * py)), TS[j]);
    ux = cadd(ux, cadd(cmul(ixi, ep), cmul(ss, es)));
    uy = cadd(uy, csub(cmul(ixi, es), cmul(sp, ep)));
  }
  double2 *o = u + ((int64_t)r * npts + ip) * 2;
  o[0] = cadd(o[0], ux);
  o[1] = cadd(o[1], uy);
}

// Adjoint of the field evaluation, g = F^H res (the right-hand side of the
// adjoint system of a receiver misfit).  Direct part, lane = particle, one
// wave type per grid z: for every receiver
//   P (alpha):  g_n += conj(d_x v_n) res_x + conj(d_y v_n) res_y,
//   S (beta):   g_n += conj(-d_y v_n) res_x + conj(d_x v_n) res_y,
// with d_x v_n = (k/2)(v_{n-1} - v_{n+1}), d_y v_n = (i k/2)(v_{n-1} + v_{n+1}).
// Receivers and residuals are staged through LDS in tiles of 256; v_k for
// k = -(PM+1)..PM+1 is swept once per (particle, receiver) with a window of
// three values.  Writes [nrhs][ncoef] (every coefficient of the wave type).
template <int PM>
__global__ __launch_bounds__(256) void field_direct_adjoint_kernel(
    int n, int npts, const double *__restrict__ xy, const int *__restrict__ p,
    const int64_t *__restrict__ off, const double *__restrict__ pts,
    const double2 *__restrict__ res, double2 *__restrict__ g, int64_t ldg, double kp, double ks) {
  constexpr int L = PM + 1;
  __shared__ double2 tp[256];      // receiver coordinates
  __shared__ double2 tr[256][2];   // residual (x, y)
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y, w = blockIdx.z;
  const int mc = m < n ? m : n - 1;
  const double xm = xy[2 * mc], ym = xy[2 * mc + 1];
  const int pm = p[mc];
  const double k = w ? ks : kp;
  const double2 *rr = res + (int64_t)r * npts * 2;
  double2 acc[2 * PM + 1];
#pragma unroll
  for (int q = 0; q < 2 * PM + 1; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int t0 = 0; t0 < npts; t0 += 256) {
    const int cnt = min(256, npts - t0);
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      const int ip = t0 + threadIdx.x;
      tp[threadIdx.x] = make_double2(pts[2 * ip], pts[2 * ip + 1]);
      tr[threadIdx.x][0] = rr[2 * ip];
      tr[threadIdx.x][1] = rr[2 * ip + 1];
    }
    __syncthreads();
    for (int t = 0; t < cnt; ++t) {
      const double dx = tp[t].x - xm, dy = tp[t].y - ym;
      const double rad = sqrt(dx * dx + dy * dy);
      const double th = atan2(dy, dx);
      double sn, cs;
      sincos(th, &sn, &cs);
      const double2 e1 = make_double2(cs, sn);
      const double z = k * rad;
      // H_0..H_L by upward recurrence (stable for the dominant Y part)
      double2 H[L + 1];
      H[0] = make_double2(j0(z), y0(z));
      H[1] = make_double2(j1(z), y1(z));
      const double iz = 2.0 / z;
#pragma unroll
      for (int q = 2; q <= L; ++q) H[q] = csub(cscale(H[q - 1], (q - 1) * iz), H[q - 2]);
      const double2 rx = tr[t][0], ry = tr[t][1];
      // phase e^{i k th} from k = -L upward
      double2 ph = make_double2(1.0, 0.0);
      const double2 em = cconj(e1);
#pragma unroll
      for (int q = 0; q < L; ++q) ph = cmul(ph, em);
      double2 va = make_double2(0.0, 0.0), vb = make_double2(0.0, 0.0);  // v_{k-2}, v_{k-1}
#pragma unroll
      for (int kk = -L; kk <= L; ++kk) {
        const int ak = kk < 0 ? -kk : kk;
        double2 vk = cmul(H[ak], ph);
        if (kk < 0 && (ak & 1)) vk = cscale(vk, -1.0);
        ph = cmul(ph, e1);
        if (kk >= -L + 2) {
          const int nn = kk - 1;  // v_{nn-1} = va, v_{nn+1} = vk
          const double2 dif = csub(va, vk), sum = cadd(va, vk);
          const double2 gx = cscale(dif, 0.5 * k);                       // d_x v_n
          const double2 gy = make_double2(-0.5 * k * sum.y, 0.5 * k * sum.x);  // d_y v_n
          double2 cxv, cyv;  // field components contributed per unit coefficient
          if (w == 0) {
            cxv = gx;
            cyv = gy;
          } else {
            cxv = make_double2(-gy.x, -gy.y);
            cyv = gx;
          }
          double2 &a = acc[nn + PM];
          a = cadd(a, cadd(cmul(cconj(cxv), rx), cmul(cconj(cyv), ry)));
        }
        va = vb;
        vb = vk;
      }
    }
  }
  if (m < n) {
    double2 *o = g + (int64_t)r * ldg + off[m] + w * (2 * pm + 1) + pm;
#pragma unroll
    for (int nn = -PM; nn <= PM; ++nn)
      if (nn >= -pm && nn <= pm) o[nn] = acc[nn + PM];
  }
}

// Adjoint of the reflected field at the nodes:
//   [RPa; RSa]_j = sum_rcv [conj(i xi e_p), conj(s_p e_p); conj(-s_s e_s), conj(i xi e_s)] res,
// written to the first chunk slot of the aggregate partials (the other slots
// are cleared), so the adjoint reflect and the adjoint disaggregate follow as
// in the adjoint operator.
__global__ __launch_bounds__(256) void field_refl_adjoint_kernel(
    int q, int npts, int chunks, const double2 *__restrict__ xi_t, const double2 *__restrict__ sp_t,
    const double2 *__restrict__ ss_t, const double *__restrict__ pts,
    const double2 *__restrict__ res, double2 *__restrict__ agg) {
  __shared__ double2 tp[256];
  __shared__ double2 tr[256][2];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  const int jc = j < q ? j : q - 1;
  const double2 xi = xi_t[jc], sp = sp_t[jc], ss = ss_t[jc];
  const double2 ixi = make_double2(-xi.y, xi.x);
  const double2 *rr = res + (int64_t)r * npts * 2;
  double2 ap = make_double2(0.0, 0.0), as = make_double2(0.0, 0.0);
  for (int t0 = 0; t0 < npts; t0 += 256) {
    const int cnt = min(256, npts - t0);
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      const int ip = t0 + threadIdx.x;
      tp[threadIdx.x] = make_double2(pts[2 * ip], pts[2 * ip + 1]);
      tr[threadIdx.x][0] = rr[2 * ip];
      tr[threadIdx.x][1] = rr[2 * ip + 1];
    }
    __syncthreads();
    for (int t = 0; t < cnt; ++t) {
      const double px = tp[t].x, py = tp[t].y;
      const double2 ep = cexp(make_double2(-xi.y * px + sp.x * py, xi.x * px + sp.y * py));
      const double2 es = cexp(make_double2(-xi.y * px + ss.x * py, xi.x * px + ss.y * py));
      const double2 rx = tr[t][0], ry = tr[t][1];
      ap = cadd(ap, cmul(cconj(ep), cadd(cmul(cconj(ixi), rx), cmul(cconj(sp), ry))));
      as = cadd(as, cmul(cconj(es), csub(cmul(cconj(ixi), ry), cmul(cconj(ss), rx))));
    }
  }
  if (j < q) {
    for (int c = 0; c < chunks; ++c) {
      agg[((int64_t)(r * 2 + 0) * chunks + c) * q + j] = c ? make_double2(0.0, 0.0) : ap;
      agg[((int64_t)(r * 2 + 1) * chunks + c) * q + j] = c ? make_double2(0.0, 0.0) : as;
    }
  }
}

#define EMS_FIELD_CASE(PMV)                                                                   \
  case PMV:                                                                                   \
    hipLaunchKernelGGL((field_direct_kernel<PMV>), grid, dim3(256), 0, st, h->n, npts, h->d_xy, \
                       h->d_p, h->d_off, gamma, h->ncoef, pts, u, h->md.kp, h->md.ks);       \
    break;

hipError_t launch_field_direct(const ems_handle *h, const double2 *gamma, int nrhs, int npts,
                               const double *pts, double2 *u, hipStream_t st) {
  dim3 grid((npts + 255) / 256, nrhs);
  switch (pm_bucket(h->pmax)) {
    EMS_FIELD_CASE(4)
    EMS_FIELD_CASE(8)
    EMS_FIELD_CASE(10)
    EMS_FIELD_CASE(12)
    EMS_FIELD_CASE(15)
    EMS_FIELD_CASE(16)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define EMS_FIELDA_CASE(PMV)                                                                  \
  case PMV:                                                                                   \
    hipLaunchKernelGGL((field_direct_adjoint_kernel<PMV>), grid, dim3(256), 0, st, h->n, npts,  \
                       h->d_xy, h->d_p, h->d_off, pts, res, g, h->ncoef, h->md.kp, h->md.ks);  \
    break;

hipError_t launch_field_direct_adjoint(const ems_handle *h, const double2 *res, int nrhs,
                                       int npts, const double *pts, double2 *g, hipStream_t st) {
  dim3 grid((h->n + 255) / 256, nrhs, 2);
  switch (pm_bucket(h->pmax)) {
    EMS_FIELDA_CASE(4)
    EMS_FIELDA_CASE(8)
    EMS_FIELDA_CASE(10)
    EMS_FIELDA_CASE(12)
    EMS_FIELDA_CASE(15)
    EMS_FIELDA_CASE(16)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_field_refl_adjoint(const ems_handle *h, const double2 *res, int nrhs, int npts,
                                     const double *pts, hipStream_t st) {
  dim3 grid((h->q + 255) / 256, nrhs);
  hipLaunchKernelGGL(field_refl_adjoint_kernel, grid, dim3(256), 0, st, h->q, npts, h->agg_chunks,
                     h->d_xi, h->d_sp, h->d_ss, pts, res, h->d_agg);
  return hipGetLastError();
}

hipError_t launch_field_trans(const ems_handle *h, int nrhs, int npts, const double *pts,
                              double2 *u, hipStream_t st) {
  dim3 grid((npts + 255) / 256, nrhs);
  hipLaunchKernelGGL(field_trans_kernel, grid, dim3(256), 0, st, h->q, npts, h->d_xi, h->d_spb,
                     h->d_ssb, h->d_refl, pts, u);
  return hipGetLastError();
}

hipError_t launch_field_refl(const ems_handle *h, int nrhs, int npts, const double *pts,
                             double2 *u, hipStream_t st) {
  dim3 grid((npts + 255) / 256, nrhs);
  hipLaunchKernelGGL(field_refl_kernel, grid, dim3(256), 0, st, h->q, npts, h->d_xi, h->d_sp,
                     h->d_ss, h->d_refl, pts, u);
  return hipGetLastError();
}

}  // namespace ems
