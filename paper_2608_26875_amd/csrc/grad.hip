// Gradient of a receiver misfit with respect to the particle centres and the
// substrate's Lame parameters (adjoint method on the Schur-complement system
// of Sections 4.2 and 5.2).
//
// Centres.  Both translation parts satisfy the same two identities, which
// follow from d_x (Z_n e^{i n th}) = (k/2)(Z_{n-1} e^{i(n-1)th} - Z_{n+1} e^{i(n+1)th})
// and d_y = (i k/2)(... + ...) for Hankel and Bessel waves, and from
// i xi (i zeta)^n = (k/2)((i zeta)^{n+1} - (i zeta)^{n-1}),
// s (i zeta)^n = (i k/2)((i zeta)^{n+1} + (i zeta)^{n-1}) for the plane waves
// of Section 5 (xi = (k/2)(zeta + 1/zeta), s = (k/2)(1/zeta - zeta)):
//  * moving a receiving centre shifts its regular expansion a:
//      D_x a_n = (k/2)(a_{n+1} - a_{n-1}),  D_y a_n = (i k/2)(a_{n+1} + a_{n-1});
//  * moving a source centre is the same operator applied to the shifted
//    source coefficients:
//      S_x c_n = (k/2)(c_{n-1} - c_{n+1}),  S_y c_n = -(i k/2)(c_{n+1} + c_{n-1}).
// With mu = S^H lambda, the incoming field a + a0 at order p + 1 and the
// adjoint sources f + z = (F^H res + T^H mu) at order p + 1 (an operator with
// orders p + 1 and S = I provides both):
//   dJ/dtheta_m = Re sum_r [ mu_m^H D_theta (a + a0)_m + (f + z)_m^H S_theta gamma_m ].
//
// Lame parameters.  Only R(xi) depends on them (and R(xi0) in the
// right-hand side):
//   dJ/dtheta = Re sum_r [ sum_j w_j Lam_j^H dR_j Ig_j + mu^H a0[dR(xi0)] ],
// Ig = (I_p / (i pi s_p), I_s / (i pi s_s)) the aggregated solution,
// Lam = C^H mu + G^H res the adjoint node amplitudes (disaggregate and
// reflected-field adjoints).
#include "dev.h"
#include "ems_internal.h"

namespace ems {

// Copy coefficient vectors between two orderings of the same particles with
// orders ps (source) and pd (destination); modes beyond ps are zero.
__global__ __launch_bounds__(128) void repack_kernel(
    const int *__restrict__ ps, const int64_t *__restrict__ offs, const int *__restrict__ pd,
    const int64_t *__restrict__ offd, const double2 *__restrict__ in, int64_t ldi,
    double2 *__restrict__ out, int64_t ldo) {
  const int m = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
  const int a = ps[m], b = pd[m];
  const int Nd = 2 * b + 1;
  if (lane >= 2 * Nd) return;
  const int w = lane / Nd, nn = lane % Nd - b;
  double2 v = make_double2(0.0, 0.0);
  if (nn >= -a && nn <= a) v = in[(int64_t)r * ldi + offs[m] + w * (2 * a + 1) + a + nn];
  out[(int64_t)r * ldo + offd[m] + lane] = v;
}

// One thread per particle: the centre gradient from the order-p vectors
// (gamma, mu) and the order-(p+1) ones (a + a0, f + z).
__global__ __launch_bounds__(256) void grad_centres_kernel(
    int n, int nrhs, const int *__restrict__ p, const int64_t *__restrict__ off,
    const int64_t *__restrict__ offe, const double2 *__restrict__ gam,
    const double2 *__restrict__ mu, int64_t ldh, const double2 *__restrict__ ae,
    const double2 *__restrict__ a0e, const double2 *__restrict__ fe,
    const double2 *__restrict__ ze, int64_t lde, double kp, double ks, double *__restrict__ dxy) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  const int pm = p[m], pe = pm + 1;
  double gx = 0.0, gy = 0.0;
  for (int r = 0; r < nrhs; ++r) {
    for (int w = 0; w < 2; ++w) {
      const double k = w ? ks : kp;
      const double2 *g = gam + (int64_t)r * ldh + off[m] + w * (2 * pm + 1) + pm;
      const double2 *u = mu + (int64_t)r * ldh + off[m] + w * (2 * pm + 1) + pm;
      const int64_t be = (int64_t)r * lde + offe[m] + w * (2 * pe + 1) + pe;
      auto A = [&](int nn) { return cadd(ae[be + nn], a0e[be + nn]); };
      auto B = [&](int nn) { return cadd(fe[be + nn], ze[be + nn]); };
      auto G = [&](int nn) { return (nn >= -pm && nn <= pm) ? g[nn] : make_double2(0.0, 0.0); };
      // target side: mu^H D a
      for (int nn = -pm; nn <= pm; ++nn) {
        const double2 ap = A(nn + 1), am = A(nn - 1);
        const double2 cu = cconj(u[nn]);
        const double2 dx = cscale(csub(ap, am), 0.5 * k);
        const double2 s = cadd(ap, am);
        const double2 dy = make_double2(-0.5 * k * s.y, 0.5 * k * s.x);
        gx += cmul(cu, dx).x;
        gy += cmul(cu, dy).x;
      }
      // source side: (f + z)^H S gamma
      for (int nn = -pe; nn <= pe; ++nn) {
        const double2 cb = cconj(B(nn));
        const double2 gp = G(nn + 1), gm = G(nn - 1);
        const double2 sx = cscale(csub(gm, gp), 0.5 * k);
        const double2 s = cadd(gp, gm);
        const double2 sy = make_double2(0.5 * k * s.y, -0.5 * k * s.x);  // -(i k/2) s
        gx += cmul(cb, sx).x;
        gy += cmul(cb, sy).x;
      }
    }
  }
  dxy[2 * m] = gx;
  dxy[2 * m + 1] = gy;
}

// Ig[r][w][j] = (sum over chunks of the aggregate) / (i pi s_w(j))
__global__ void lame_ig_kernel(int q, int chunks, const double2 *__restrict__ agg,
                               const double2 *__restrict__ sp_t, const double2 *__restrict__ ss_t,
                               double2 *__restrict__ Ig) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (j >= q) return;
  const double kInvPi = 0.31830988618379067154;
  for (int w = 0; w < 2; ++w) {
    double2 I = make_double2(0.0, 0.0);
    for (int c = 0; c < chunks; ++c) I = cadd(I, agg[((int64_t)(r * 2 + w) * chunks + c) * q + j]);
    const double2 s = w ? ss_t[j] : sp_t[j];
    const double d = s.x * s.x + s.y * s.y;
    const double2 cf = make_double2(-s.y * kInvPi / d, -s.x * kInvPi / d);  // 1/(i pi s)
    Ig[(int64_t)(r * 2 + w) * q + j] = cmul(I, cf);
  }
}

// Lam[r][w][j] (+)= sum over chunks of the aggregate slots
__global__ void lame_lam_kernel(int q, int chunks, const double2 *__restrict__ agg,
                                double2 *__restrict__ Lam, int accumulate) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (j >= q) return;
  for (int w = 0; w < 2; ++w) {
    double2 v = make_double2(0.0, 0.0);
    for (int c = 0; c < chunks; ++c) v = cadd(v, agg[((int64_t)(r * 2 + w) * chunks + c) * q + j]);
    double2 *o = Lam + (int64_t)(r * 2 + w) * q + j;
    *o = accumulate ? cadd(*o, v) : v;
  }
}

// Partial sums (per block) of Re sum_j w_j Lam_j^H dR_theta,j Ig_j, theta = lambda_b, mu_b.
__global__ __launch_bounds__(256) void lame_reduce_kernel(
    int q, int nrhs, const double2 *__restrict__ w_t, const double2 *__restrict__ dR,
    const double2 *__restrict__ Ig, const double2 *__restrict__ Lam, double *__restrict__ part) {
  __shared__ double sh[2][256];
  double t0 = 0.0, t1 = 0.0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < q; j += gridDim.x * blockDim.x) {
    const double2 wj = w_t[j];
    for (int r = 0; r < nrhs; ++r) {
      const double2 ip = Ig[(int64_t)(r * 2 + 0) * q + j], is = Ig[(int64_t)(r * 2 + 1) * q + j];
      const double2 lp = cconj(Lam[(int64_t)(r * 2 + 0) * q + j]);
      const double2 ls = cconj(Lam[(int64_t)(r * 2 + 1) * q + j]);
      for (int th = 0; th < 2; ++th) {
        const double2 *D = dR + 8 * (int64_t)j + 4 * th;
        const double2 vp = cadd(cmul(D[0], ip), cmul(D[1], is));
        const double2 vs = cadd(cmul(D[2], ip), cmul(D[3], is));
        const double v = cmul(wj, cadd(cmul(lp, vp), cmul(ls, vs))).x;
        if (th == 0) t0 += v;
        else t1 += v;
      }
    }
  }
  sh[0][threadIdx.x] = t0;
  sh[1][threadIdx.x] = t1;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sh[0][0];
    part[2 * blockIdx.x + 1] = sh[1][0];
  }
}

// Partial sums (per block) of Re sum_i conj(a_i) b_i.
__global__ __launch_bounds__(256) void re_dot_kernel(int64_t len, const double2 *__restrict__ a,
                                                     const double2 *__restrict__ b,
                                                     double *__restrict__ part) {
  __shared__ double sh[256];
  double t = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x)
    t += a[i].x * b[i].x + a[i].y * b[i].y;
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

hipError_t launch_repack(const ems_handle *src, const ems_handle *dst, const double2 *in,
                         double2 *out, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(repack_kernel, dim3(src->n, nrhs), dim3(128), 0, st, src->d_p, src->d_off,
                     dst->d_p, dst->d_off, in, src->ncoef, out, dst->ncoef);
  return hipGetLastError();
}

hipError_t launch_grad_centres(const ems_handle *h, const ems_handle *e, const double2 *gam,
                               const double2 *mu, const double2 *ae, const double2 *a0e,
                               const double2 *fe, const double2 *ze, int nrhs, double *dxy,
                               hipStream_t st) {
  hipLaunchKernelGGL(grad_centres_kernel, dim3((h->n + 255) / 256), dim3(256), 0, st, h->n, nrhs,
                     h->d_p, h->d_off, e->d_off, gam, mu, h->ncoef, ae, a0e, fe, ze, e->ncoef,
                     h->md.kp, h->md.ks, dxy);
  return hipGetLastError();
}

hipError_t launch_lame_ig(const ems_handle *h, int nrhs, double2 *Ig, hipStream_t st) {
  hipLaunchKernelGGL(lame_ig_kernel, dim3((h->q + 255) / 256, nrhs), dim3(256), 0, st, h->q,
                     h->agg_chunks, h->d_agg, h->d_sp, h->d_ss, Ig);
  return hipGetLastError();
}

hipError_t launch_lame_lam(const ems_handle *h, int nrhs, double2 *Lam, bool accumulate,
                           hipStream_t st) {
  hipLaunchKernelGGL(lame_lam_kernel, dim3((h->q + 255) / 256, nrhs), dim3(256), 0, st, h->q,
                     h->agg_chunks, h->d_agg, Lam, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_lame_reduce(const ems_handle *h, int nrhs, const double2 *Ig,
                              const double2 *Lam, double *part, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(lame_reduce_kernel, dim3(blocks), dim3(256), 0, st, h->q, nrhs, h->d_w,
                     h->d_dR, Ig, Lam, part);
  return hipGetLastError();
}

hipError_t launch_re_dot(int64_t len, const double2 *a, const double2 *b, double *part,
                         int blocks, hipStream_t st) {
  hipLaunchKernelGGL(re_dot_kernel, dim3(blocks), dim3(256), 0, st, len, a, b, part);
  return hipGetLastError();
}

}  // namespace ems
