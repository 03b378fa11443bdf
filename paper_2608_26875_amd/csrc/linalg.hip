// S-matrix apply and the final combination of the operator (Sections 4.2 and
// 5.2: y_m = x_m - S_m (T_free x + T_refl x)_m), the plane-wave right-hand
// side (Section 7.3), and the vector kernels of the GMRES driver.
//
// The S store is packed per particle column-major (S^T row-major), so the
// 4p+2 lanes of one wavefront read one column of S_m in a single coalesced
// 16-byte-per-lane transaction while the input coefficient is broadcast from
// LDS.
#include "dev.h"
#include "ems_internal.h"

namespace ems {

__device__ __forceinline__ double2 to_c128(double2 v) { return v; }
__device__ __forceinline__ double2 to_c128(float2 v) { return make_double2(v.x, v.y); }

// One workgroup per particle (64 or 128 lanes); lane = row of the particle block.
// SC: the S store read, complex128, or its complex64 copy for the mixed form
// (half the bytes of the kernel's largest stream; products accumulate in FP64).
// DC: the disaggregate's partial sums (complex64 from the FP32 kernel).
template <typename SC, typename DC>
__global__ __launch_bounds__(128) void combine_kernel(
    const int *__restrict__ p, const int64_t *__restrict__ off,
    const int64_t *__restrict__ Soff, const SC *__restrict__ St,
    const double2 *__restrict__ x, double2 *__restrict__ y, const double2 *__restrict__ fre,
    const DC *__restrict__ dis, int chunks, int64_t ncoef, int flags, int sign) {
  __shared__ double2 v[2 * kMaxModes];
  const int m = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
  const int pm = p[m];
  const int N = 2 * pm + 1, K = 2 * N;
  const int64_t base = (int64_t)r * ncoef + off[m];
  if (lane < K) {
    double2 val = make_double2(0.0, 0.0);
    if (flags & EMS_PART_FREE) val = fre[base + lane];
    if (flags & EMS_PART_REFL) {
      double2 s = make_double2(0.0, 0.0);
      const DC *dr = dis + (int64_t)r * chunks * ncoef + off[m] + lane;
      for (int c = 0; c < chunks; ++c) s = cadd(s, to_c128(dr[(int64_t)c * ncoef]));
      const int nn = (lane < N ? lane : lane - N) - pm;
      if (sign && (nn & 1)) s = cscale(s, -1.0);
      val = cadd(val, s);
    }
    v[lane] = val;
  }
  __syncthreads();
  if (lane < K) {
    double2 u;
    if (flags & EMS_PART_S) {
      u = make_double2(0.0, 0.0);
      const SC *Sm = St + Soff[m];
      for (int c = 0; c < K; ++c) cfma(u, to_c128(Sm[(int64_t)c * K + lane]), v[c]);
    } else {
      u = v[lane];
    }
    if (flags & EMS_PART_IDENTITY) u = csub(x[base + lane], u);
    y[base + lane] = u;
  }
}

// y_m = S_m c_m (adjoint = 0) or S_m^H c_m (adjoint = 1)
__global__ __launch_bounds__(128) void s_apply_kernel(
    const int *__restrict__ p, const int64_t *__restrict__ off,
    const int64_t *__restrict__ Soff, const double2 *__restrict__ St,
    const double2 *__restrict__ c, double2 *__restrict__ y, int64_t ncoef, int adjoint) {
  __shared__ double2 v[2 * kMaxModes];
  const int m = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
  const int pm = p[m];
  const int K = 2 * (2 * pm + 1);
  const int64_t base = (int64_t)r * ncoef + off[m];
  if (lane < K) v[lane] = c[base + lane];
  __syncthreads();
  if (lane < K) {
    double2 u = make_double2(0.0, 0.0);
    const double2 *Sm = St + Soff[m];
    if (!adjoint) {
      for (int k = 0; k < K; ++k) cfma(u, Sm[(int64_t)k * K + lane], v[k]);
    } else {
      for (int k = 0; k < K; ++k) cfma(u, cconj(Sm[(int64_t)lane * K + k]), v[k]);
    }
    y[base + lane] = u;
  }
}

hipError_t launch_combine(const ems_handle *h, const double2 *x, double2 *y, int nrhs, int flags,
                          bool adjoint, bool mixed, hipStream_t st) {
  const dim3 grid(h->n, nrhs), block(part_threads(h));
  const int sg = adjoint ? 0 : 1;
  // the partials' type follows the kernel that wrote them; S independently
  const bool s32 = mixed && h->d_S32, d32 = somm_dis_c64(h, adjoint, mixed);
  const float2 *dis32 = reinterpret_cast<const float2 *>(h->d_dis);
#define EMS_COMBINE(SC, DC, S, D)                                                               \
  hipLaunchKernelGGL((combine_kernel<SC, DC>), grid, block, 0, st, h->d_p, h->d_off, h->d_Soff, \
                     S, x, y, h->d_free, D, h->dis_chunks, h->ncoef, flags, sg)
  if (s32 && d32) EMS_COMBINE(float2, float2, h->d_S32, dis32);
  else if (s32) EMS_COMBINE(float2, double2, h->d_S32, h->d_dis);
  else if (d32) EMS_COMBINE(double2, float2, h->d_S, dis32);
  else EMS_COMBINE(double2, double2, h->d_S, h->d_dis);
#undef EMS_COMBINE
  return hipGetLastError();
}

hipError_t launch_s_apply(const ems_handle *h, const double2 *c, double2 *y, int nrhs,
                          bool adjoint, hipStream_t st) {
  hipLaunchKernelGGL(s_apply_kernel, dim3(h->n, nrhs), dim3(part_threads(h)), 0, st, h->d_p, h->d_off,
                     h->d_Soff, h->d_S, c, y, h->ncoef, adjoint ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_s_multiply(const ems_handle *h, const double2 *c, double2 *y, int nrhs,
                             hipStream_t st) {
  return launch_s_apply(h, c, y, nrhs, false, st);
}

// ---------------------------------------------------------------------------
// Plane-wave local coefficients (Section 7.3 background field; Jacobi-Anger).
// Per right-hand side r the host supplies pw[r] = {xi0, s_p, s_s, Ain_p,
// Ain_s, Ar_p, Ar_s} (complex), and
//   a_n = Ar_p e^{i xi0 x + s_p y} (i (xi0 - s_p)/kp)^n + Ain_p e^{i xi0 x - s_p y} (i (xi0 + s_p)/kp)^n
//   b_n = the same with (s_s, ks, Ar_s, Ain_s).
__device__ double2 cpow_int(double2 z, int n) {
  double2 r = make_double2(1.0, 0.0);
  const int an = n < 0 ? -n : n;
  for (int k = 0; k < an; ++k) r = cmul(r, z);
  if (n < 0) {
    const double d = r.x * r.x + r.y * r.y;
    r = make_double2(r.x / d, -r.y / d);
  }
  return r;
}

__global__ void incident_kernel(int n, const double *__restrict__ xy, const int *__restrict__ p,
                                 const int64_t *__restrict__ off, const double2 *__restrict__ pw,
                                 double kp, double ks, double2 *__restrict__ c, int64_t ncoef) {
  const int m = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
  const int pm = p[m];
  const int N = 2 * pm + 1;
  if (lane >= 2 * N) return;
  const int wave = lane < N ? 0 : 1;
  const int nn = (wave ? lane - N : lane) - pm;
  const double2 *P = pw + 7 * r;
  const double2 xi0 = P[0];
  const double2 s = wave ? P[2] : P[1];
  const double2 Ain = wave ? P[4] : P[3];
  const double2 Ar = wave ? P[6] : P[5];
  const double k = wave ? ks : kp;
  const double x = xy[2 * m], y = xy[2 * m + 1];
  const double2 I = make_double2(0.0, 1.0);
  const double2 ixi = cmul(I, xi0);
  // reflected: e^{i xi0 x + s y} (i (xi0 - s)/k)^n
  const double2 er = cexp(cadd(cscale(ixi, x), cscale(s, y)));
  const double2 br = cscale(cmul(I, csub(xi0, s)), 1.0 / k);
  const double2 ei = cexp(csub(cscale(ixi, x), cscale(s, y)));
  const double2 bi = cscale(cmul(I, cadd(xi0, s)), 1.0 / k);
  double2 v = cmul(cmul(Ar, er), cpow_int(br, nn));
  v = cadd(v, cmul(cmul(Ain, ei), cpow_int(bi, nn)));
  c[(int64_t)r * ncoef + off[m] + lane] = v;
}

hipError_t launch_incident_pw(const ems_handle *h, const double2 *pw, int nrhs, double2 *c,
                              hipStream_t st) {
  hipLaunchKernelGGL(incident_kernel, dim3(h->n, nrhs), dim3(part_threads(h)), 0, st, h->n, h->d_xy, h->d_p,
                     h->d_off, pw, h->md.kp, h->md.ks, c, h->ncoef);
  return hipGetLastError();
}

// Point source in the substrate (Section 3.2): local expansions of its field
// transmitted into the host, over a node list of its own.  nd [q][3] = (xi,
// s_p, s_s); amp [nrhs][q][2] = w_j (Td A_inc)_{P,S}, the host's downgoing
// potentials per node (weights, e^{-i xi x0} and the source's depth factor
// included).  Local coefficient of particle m, wave w, order n:
//   sum_j amp_w(j) e^{i xi_j x_m + s_w y_m} (i (xi_j - s_w)/k_w)^n  (Jacobi-Anger).
// The powers are node quantities: point_pow_kernel tabulates them once per
// call, V [q][2][2 pmax + 1] (negative orders as the reciprocal of the
// positive power).  point_local_kernel: a block holds G groups of L lanes
// (lane = wave, order), each lane serving kPtR particles; per tile of kPtTile
// nodes the powers and the G kPtR x 2 exponentials go to LDS once, and a
// lane's power read serves its kPtR particles.
constexpr int kPtTile = 32;
constexpr int kPtLanes = 512;
constexpr int kPtR = 2;
__global__ void point_pow_kernel(int q, int pmax, const double2 *__restrict__ nd, double kp,
                                 double ks, double2 *__restrict__ V) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 2 * q) return;
  const int j = id >> 1, w = id & 1;
  const double2 xi = nd[3 * (int64_t)j], s = nd[3 * (int64_t)j + 1 + w];
  const double k = w ? ks : kp;
  const double2 d = csub(xi, s);
  const double2 z = make_double2(-d.y / k, d.x / k);   // i (xi - s) / k
  const int NP = 2 * pmax + 1;
  double2 *out = V + (int64_t)id * NP + pmax;
  double2 r = make_double2(1.0, 0.0);
  out[0] = r;
  for (int n = 1; n <= pmax; ++n) {
    r = cmul(r, z);
    out[n] = r;
    const double dd = r.x * r.x + r.y * r.y;
    out[-n] = make_double2(r.x / dd, -r.y / dd);
  }
}

__global__ __launch_bounds__(kPtLanes) void point_local_kernel(
    int n, int q, int pmax, int L, const double *__restrict__ xy, const int *__restrict__ p,
    const int64_t *__restrict__ off, const double2 *__restrict__ nd,
    const double2 *__restrict__ amp, const double2 *__restrict__ V, double2 *__restrict__ c,
    int64_t ncoef) {
  __shared__ double2 sv[2 * kPtTile * kMaxModes];
  __shared__ double2 se[(kPtLanes / 64) * kPtR * 2 * kPtTile];
  const int G = kPtLanes / L;
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  const int mb = blockIdx.x * G * kPtR, r = blockIdx.y;
  const int NP = 2 * pmax + 1;
  // the kPtR particles of a lane: mb + rr G + g; they share the lane's order
  // only when their orders agree, so each keeps its own (wave, column)
  int mm[kPtR], colr[kPtR], wv[kPtR];
  bool act[kPtR];
#pragma unroll
  for (int rr = 0; rr < kPtR; ++rr) {
    mm[rr] = mb + rr * G + g;
    const int pm = mm[rr] < n ? p[mm[rr]] : 0;
    const int N = 2 * pm + 1;
    act[rr] = mm[rr] < n && lane < 2 * N;
    wv[rr] = lane < N ? 0 : 1;
    colr[rr] = (wv[rr] ? lane - N : lane) - pm + pmax;
  }
  const bool same = kPtR == 1 || (wv[0] == wv[kPtR - 1] && colr[0] == colr[kPtR - 1]);
  const double2 *A = amp + (int64_t)r * q * 2;
  double2 acc[kPtR];
#pragma unroll
  for (int rr = 0; rr < kPtR; ++rr) acc[rr] = make_double2(0.0, 0.0);
  for (int j0 = 0; j0 < q; j0 += kPtTile) {
    const int tn = min(kPtTile, q - j0);
    // powers of the tile: contiguous [t][w][order] block of V
    for (int e = threadIdx.x; e < tn * 2 * NP; e += kPtLanes) sv[e] = V[(int64_t)j0 * 2 * NP + e];
    // exponentials amp_w(j) e^{i xi x_m + s_w y_m}, one per (particle, wave, node)
    for (int e = threadIdx.x; e < G * kPtR * 2 * kPtTile; e += kPtLanes) {
      const int gg = e / (2 * kPtTile), rem = e % (2 * kPtTile), w = rem / kPtTile,
                tt = rem % kPtTile;
      const int mp = mb + gg;   // block particle gg = rr G + g
      double2 v = make_double2(0.0, 0.0);
      if (mp < n && tt < tn) {
        const int j = j0 + tt;
        const double x = xy[2 * mp], y = xy[2 * mp + 1];
        const double2 xi = nd[3 * (int64_t)j], s = nd[3 * (int64_t)j + 1 + w];
        v = cmul(A[2 * (int64_t)j + w],
                 cexp(make_double2(-xi.y * x + s.x * y, xi.x * x + s.y * y)));
      }
      se[e] = v;
    }
    __syncthreads();
    // equal (wave, column) means equal orders, hence the same activity
    if (same) {
      if (act[0]) {
        // one power read per node for all kPtR particles of the lane
        const double2 *pv = sv + wv[0] * NP + colr[0];
        for (int t = 0; t < tn; ++t) {
          const double2 vp = pv[t * 2 * NP];
#pragma unroll
          for (int rr = 0; rr < kPtR; ++rr)
            cfma(acc[rr], se[((rr * G + g) * 2 + wv[0]) * kPtTile + t], vp);
        }
      }
    } else {
#pragma unroll
      for (int rr = 0; rr < kPtR; ++rr) {
        if (act[rr]) {
          const double2 *ev = se + ((rr * G + g) * 2 + wv[rr]) * kPtTile;
          const double2 *pv = sv + wv[rr] * NP + colr[rr];
          for (int t = 0; t < tn; ++t) cfma(acc[rr], ev[t], pv[t * 2 * NP]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int rr = 0; rr < kPtR; ++rr)
    if (act[rr]) c[(int64_t)r * ncoef + off[mm[rr]] + lane] = acc[rr];
}

hipError_t launch_point_local(const ems_handle *h, int q, const double2 *nd, const double2 *amp,
                              int nrhs, double2 *c, double2 *V, hipStream_t st) {
  const int pmax = h->pmax;
  hipLaunchKernelGGL(point_pow_kernel, dim3((2 * q + 255) / 256), dim3(256), 0, st, q, pmax, nd,
                     h->md.kp, h->md.ks, V);
  const int L = part_threads(h), G = kPtLanes / L;
  hipLaunchKernelGGL(point_local_kernel, dim3((h->n + G * kPtR - 1) / (G * kPtR), nrhs),
                     dim3(kPtLanes), 0, st,
                     h->n, q, pmax, L, h->d_xy, h->d_p, h->d_off, nd, amp, V, c, h->ncoef);
  return hipGetLastError();
}

// Background displacement of point sources at receivers of either layer.
// Host (y < 0): the transmitted potentials amp_h = w (Td A_inc) on e^{i xi x
// + s y}; substrate (y > 0): the Green's tensor (closed form, Hankel
// functions of the substrate's wavenumbers) plus the reflected potentials
// amp_b = w (Rb A_inc) on e^{i xi x - s_b y}.  nd [q][5] = (xi, s_p, s_s,
// s_pb, s_sb); amp [nrhs][q][4] = (amp_h P, S, amp_b P, S); src [nrhs][4] =
// (x0, y0, alpha1, alpha2).
__global__ void point_field_kernel(int npts, int q, const double *__restrict__ pts,
                                   const double2 *__restrict__ nd, const double2 *__restrict__ amp,
                                   const double *__restrict__ src, double kpb, double ksb,
                                   double inv_rw2, double2 *__restrict__ u) {
  const int ip = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (ip >= npts) return;
  const double x = pts[2 * ip], y = pts[2 * ip + 1];
  const bool host = y < 0.0;
  const double2 *A = amp + (int64_t)r * q * 4 + (host ? 0 : 2);
  double2 ux = make_double2(0.0, 0.0), uy = make_double2(0.0, 0.0);
  for (int j = 0; j < q; ++j) {
    const double2 xi = nd[5 * (int64_t)j];
    const double2 ixi = make_double2(-xi.y, xi.x);
    // P: q = +s_p (host) or -s_pb (substrate); S likewise
    double2 qp = nd[5 * (int64_t)j + (host ? 1 : 3)];
    double2 qs = nd[5 * (int64_t)j + (host ? 2 : 4)];
    if (!host) {
      qp = cscale(qp, -1.0);
      qs = cscale(qs, -1.0);
    }
    const double2 ep = cmul(A[4 * (int64_t)j], cexp(make_double2(-xi.y * x + qp.x * y, xi.x * x + qp.y * y)));
    const double2 es = cmul(A[4 * (int64_t)j + 1], cexp(make_double2(-xi.y * x + qs.x * y, xi.x * x + qs.y * y)));
    // grad (i xi, q) and grad^perp (-q, i xi)
    ux = cadd(ux, csub(cmul(ixi, ep), cmul(qs, es)));
    uy = cadd(uy, cadd(cmul(qp, ep), cmul(ixi, es)));
  }
  if (!host) {
    // Green's tensor 1/(rho w^2) (ks^2 g_s I + grad grad^T (g_s - g_p)) alpha,
    // g = (i/4) H0(k r); d_i d_j g = (i/4) k^2 [d2 e_i e_j + (d1 / z)(delta_ij - e_i e_j)],
    // d1 = -H1(z), d2 = -H0(z) + H1(z)/z
    const double *S = src + 4 * r;
    const double dx = x - S[0], dy = y - S[1];
    const double rr = sqrt(dx * dx + dy * dy);
    const double ex = dx / rr, ey = dy / rr;
    const double a1 = S[2], a2 = S[3];
    const double ea = ex * a1 + ey * a2;
    double2 gx = make_double2(0.0, 0.0), gy = make_double2(0.0, 0.0);
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const double k = w ? kpb : ksb;
      const double sg = w ? -1.0 : 1.0;
      const double z = k * rr;
      const double2 h0 = make_double2(j0(z), y0(z)), h1 = make_double2(j1(z), y1(z));
      const double2 d1 = cscale(h1, -1.0);
      const double2 d2 = cadd(cscale(h0, -1.0), cscale(h1, 1.0 / z));
      // (i/4) k^2 [d2 (e.a) e + (d1/z)(a - (e.a) e)]
      const double2 f = cscale(make_double2(0.0, 0.25), sg * k * k);
      const double2 cx = cadd(cscale(d2, ea * ex), cscale(d1, (a1 - ea * ex) / z));
      const double2 cy = cadd(cscale(d2, ea * ey), cscale(d1, (a2 - ea * ey) / z));
      gx = cadd(gx, cmul(f, cx));
      gy = cadd(gy, cmul(f, cy));
      if (w == 0) {
        // ks^2 g_s alpha
        const double2 g = cmul(make_double2(0.0, 0.25 * k * k), h0);
        gx = cadd(gx, cscale(g, a1));
        gy = cadd(gy, cscale(g, a2));
      }
    }
    ux = cadd(ux, cscale(gx, inv_rw2));
    uy = cadd(uy, cscale(gy, inv_rw2));
  }
  double2 *o = u + ((int64_t)r * npts + ip) * 2;
  o[0] = ux;
  o[1] = uy;
}

hipError_t launch_point_field(const ems_handle *h, int q, const double2 *nd, const double2 *amp,
                              const double *src, int nrhs, int npts, const double *pts,
                              double2 *u, hipStream_t st) {
  const double inv_rw2 = 1.0 / (h->md.rho_b * h->md.omega * h->md.omega);
  hipLaunchKernelGGL(point_field_kernel, dim3((npts + 255) / 256, nrhs), dim3(256), 0, st, npts,
                     q, pts, nd, amp, src, h->md.kpb, h->md.ksb, inv_rw2, u);
  return hipGetLastError();
}

// Background displacement of plane waves at receivers of either layer.
// comp [nrhs][6][3]: per component {A, q, (xi0, code)}, the potential
// A e^{i xi0 x + q y}; code = 2 layer + kind (layer 0 host y < 0, 1
// substrate y > 0; kind 0 P: grad -> (i xi0, q), kind 1 S: grad^perp ->
// (-q, i xi0)), code < 0 an unused slot.
__global__ void background_kernel(int npts, const double *__restrict__ pts,
                                  const double2 *__restrict__ comp, double2 *__restrict__ u) {
  const int ip = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (ip >= npts) return;
  const double x = pts[2 * ip], y = pts[2 * ip + 1];
  const int layer = y < 0.0 ? 0 : 1;
  double2 ux = make_double2(0.0, 0.0), uy = make_double2(0.0, 0.0);
  for (int c = 0; c < 6; ++c) {
    const double2 *C = comp + ((int64_t)r * 6 + c) * 3;
    const int code = (int)C[2].y;
    if (code < 0 || (code >> 1) != layer) continue;
    const double2 q = C[1];
    const double2 ixi = make_double2(0.0, C[2].x);
    const double2 e = cmul(C[0], cexp(make_double2(q.x * y, C[2].x * x + q.y * y)));
    if ((code & 1) == 0) {
      ux = cadd(ux, cmul(ixi, e));
      uy = cadd(uy, cmul(q, e));
    } else {
      ux = csub(ux, cmul(q, e));
      uy = cadd(uy, cmul(ixi, e));
    }
  }
  double2 *o = u + ((int64_t)r * npts + ip) * 2;
  o[0] = ux;
  o[1] = uy;
}

hipError_t launch_background(int nrhs, int npts, const double *pts, const double2 *comp,
                             double2 *u, hipStream_t st) {
  hipLaunchKernelGGL(background_kernel, dim3((npts + 255) / 256, nrhs), dim3(256), 0, st, npts,
                     pts, comp, u);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// GMRES vector kernels.  Reductions write one partial per block and are
// finished by a single-block kernel in a fixed order (reproducible).

__device__ __forceinline__ double2 warp_reduce(double2 v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_down(v.x, o, 64);
    v.y += __shfl_down(v.y, o, 64);
  }
  return v;
}

__device__ double2 block_reduce(double2 v) {
  __shared__ double2 sh[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = warp_reduce(v);
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double2 r = make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r = cadd(r, sh[k]);
  }
  __syncthreads();
  return r;
}

// Basis element types of GMRES: complex128, or complex64 for the inner solves
// of the mixed refinement (values are widened to FP64 on load).
__device__ __forceinline__ double2 wide(double2 v) { return v; }
__device__ __forceinline__ double2 wide(float2 v) { return make_double2((double)v.x, (double)v.y); }

// partial[i][b] = sum_{rows in block b's stripe} conj(V_i[row]) w[row] for
// MV consecutive basis vectors i per workgroup: w is read once for all of
// them and one reduction serves MV sums.
constexpr int kMdotV = 8;
template <typename TB>
__global__ __launch_bounds__(256) void mdot_kernel(const TB *__restrict__ V, int64_t ldv, int k,
                                                  const double2 *__restrict__ w, int64_t n,
                                                  double2 *__restrict__ part) {
  const int i0 = blockIdx.y * kMdotV;
  const int nv = min(kMdotV, k - i0);
  double2 acc[kMdotV];
#pragma unroll
  for (int v = 0; v < kMdotV; ++v) acc[v] = make_double2(0.0, 0.0);
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x) {
    const double2 wr = w[row];
#pragma unroll
    for (int v = 0; v < kMdotV; ++v)
      if (v < nv) cfma(acc[v], cconj(wide(V[(int64_t)(i0 + v) * ldv + row])), wr);
  }
  __shared__ double2 sh[kMdotV][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < kMdotV; ++v) {
    const double2 r = warp_reduce(acc[v]);
    if (lane == 0) sh[v][wid] = r;
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    const int v = threadIdx.x;
    double2 r = make_double2(0.0, 0.0);
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) r = cadd(r, sh[v][q]);
    part[(int64_t)(i0 + v) * gridDim.x + blockIdx.x] = r;
  }
}

__global__ void finish_kernel(const double2 *__restrict__ part, int nb, int k,
                              double2 *__restrict__ out) {
  const int i = blockIdx.x;
  double2 acc = make_double2(0.0, 0.0);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc = cadd(acc, part[(int64_t)i * nb + b]);
  acc = block_reduce(acc);
  if (threadIdx.x == 0) out[i] = acc;
}

template <typename TB>
static hipError_t mdot_go(const TB *V, int64_t ldv, int k, const double2 *w, int64_t n,
                          double2 *out_dev, double *scratch, hipStream_t st) {
  double2 *part = reinterpret_cast<double2 *>(scratch);
  hipLaunchKernelGGL(mdot_kernel<TB>, dim3(kRedBlocks, (k + kMdotV - 1) / kMdotV), dim3(256), 0,
                     st, V, ldv, k, w, n, part);
  hipLaunchKernelGGL(finish_kernel, dim3(k), dim3(256), 0, st, part, kRedBlocks, k, out_dev);
  return hipGetLastError();
}
hipError_t launch_mdot(const double2 *V, int64_t ldv, int k, const double2 *w, int64_t n,
                       double2 *out_dev, double *scratch, hipStream_t st) {
  return mdot_go(V, ldv, k, w, n, out_dev, scratch, st);
}
hipError_t launch_mdot(const float2 *V, int64_t ldv, int k, const double2 *w, int64_t n,
                       double2 *out_dev, double *scratch, hipStream_t st) {
  return mdot_go(V, ldv, k, w, n, out_dev, scratch, st);
}

// w -= sum_i V_i c_i  (c on device)
template <typename TB>
__global__ __launch_bounds__(256) void mupdate_kernel(const TB *__restrict__ V, int64_t ldv,
                                                     int k, const double2 *__restrict__ c,
                                                     double2 *__restrict__ w, int64_t n,
                                                     double sgn) {
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x) {
    double2 acc = make_double2(0.0, 0.0);
    for (int i = 0; i < k; ++i) cfma(acc, wide(V[(int64_t)i * ldv + row]), c[i]);
    w[row] = make_double2(w[row].x + sgn * acc.x, w[row].y + sgn * acc.y);
  }
}

template <typename TB>
static hipError_t mupdate_go(const TB *V, int64_t ldv, int k, const double2 *c, double2 *w,
                             int64_t n, double sgn, hipStream_t st) {
  hipLaunchKernelGGL(mupdate_kernel<TB>, dim3(2048), dim3(256), 0, st, V, ldv, k, c, w, n, sgn);
  return hipGetLastError();
}
hipError_t launch_mupdate(const double2 *V, int64_t ldv, int k, const double2 *c, double2 *w,
                          int64_t n, hipStream_t st) {
  return mupdate_go(V, ldv, k, c, w, n, -1.0, st);
}
hipError_t launch_mupdate(const float2 *V, int64_t ldv, int k, const double2 *c, double2 *w,
                          int64_t n, hipStream_t st) {
  return mupdate_go(V, ldv, k, c, w, n, -1.0, st);
}
hipError_t launch_maccum(const double2 *V, int64_t ldv, int k, const double2 *c, double2 *y,
                         int64_t n, hipStream_t st) {
  return mupdate_go(V, ldv, k, c, y, n, 1.0, st);
}
hipError_t launch_maccum(const float2 *V, int64_t ldv, int k, const double2 *c, double2 *y,
                         int64_t n, hipStream_t st) {
  return mupdate_go(V, ldv, k, c, y, n, 1.0, st);
}

// Narrowing and widening copies between the FP64 vectors and an FP32 basis.
__global__ void copy_scaled_f32_kernel(const double2 *src, float2 *dst, int64_t n, double s) {
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x)
    dst[row] = make_float2((float)(s * src[row].x), (float)(s * src[row].y));
}
__global__ void widen_kernel(const float2 *src, double2 *dst, int64_t n) {
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x)
    dst[row] = wide(src[row]);
}
hipError_t launch_copy_scaled(const double2 *src, float2 *dst, int64_t n, double s,
                              hipStream_t st) {
  hipLaunchKernelGGL(copy_scaled_f32_kernel, dim3(2048), dim3(256), 0, st, src, dst, n, s);
  return hipGetLastError();
}
hipError_t launch_widen(const float2 *src, double2 *dst, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(widen_kernel, dim3(2048), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void norm2_kernel(const double2 *__restrict__ w, int64_t n,
                                                   double2 *__restrict__ part) {
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = w[row];
    acc.x = fma(v.x, v.x, fma(v.y, v.y, acc.x));
  }
  acc = block_reduce(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void finish_norm_kernel(const double2 *__restrict__ part, int nb, double *out) {
  double2 acc = make_double2(0.0, 0.0);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc = cadd(acc, part[b]);
  acc = block_reduce(acc);
  if (threadIdx.x == 0) out[0] = sqrt(acc.x);
}

hipError_t launch_norm2(const double2 *w, int64_t n, double *out_dev, double *scratch,
                        hipStream_t st) {
  double2 *part = reinterpret_cast<double2 *>(scratch);
  hipLaunchKernelGGL(norm2_kernel, dim3(kRedBlocks), dim3(256), 0, st, w, n, part);
  hipLaunchKernelGGL(finish_norm_kernel, dim3(1), dim3(256), 0, st, part, kRedBlocks, out_dev);
  return hipGetLastError();
}

__global__ void scale_kernel(double2 *w, int64_t n, double s) {
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x)
    w[row] = cscale(w[row], s);
}
__global__ void copy_scaled_kernel(const double2 *src, double2 *dst, int64_t n, double s) {
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x)
    dst[row] = cscale(src[row], s);
}
__global__ void axpy_kernel(double2 *y, const double2 *x, int64_t n, double a) {
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x)
    y[row] = make_double2(y[row].x + a * x[row].x, y[row].y + a * x[row].y);
}

hipError_t launch_scale(double2 *w, int64_t n, double s, hipStream_t st) {
  hipLaunchKernelGGL(scale_kernel, dim3(2048), dim3(256), 0, st, w, n, s);
  return hipGetLastError();
}
hipError_t launch_copy_scaled(const double2 *src, double2 *dst, int64_t n, double s,
                              hipStream_t st) {
  hipLaunchKernelGGL(copy_scaled_kernel, dim3(2048), dim3(256), 0, st, src, dst, n, s);
  return hipGetLastError();
}
hipError_t launch_axpy(double2 *y, const double2 *x, int64_t n, double a, hipStream_t st) {
  hipLaunchKernelGGL(axpy_kernel, dim3(2048), dim3(256), 0, st, y, x, n, a);
  return hipGetLastError();
}

}  // namespace ems
