// Scattering matrices of non-circular particles (Section 4.3), generated on
// the GPU, one particle per workgroup, by the method of fundamental
// solutions: the scattered field of a particle is carried by N compressional
// and N shear monopoles H_0(k |x - y_j|) at sources y_j = z(t_j + i delta)
// (the boundary parametrisation continued inward), and the boundary
// condition (rigid: u = -u_inc; traction-free: sigma.nu = -sigma_inc.nu) is
// collocated at the N boundary points z(t_j).  With the incident basis
// grad(J_n(kp r) e^{i n th}), grad^perp(J_n(ks r) e^{i n th}), n = -p..p, as
// right-hand sides, the 2N x 2N system is solved for 2(2p+1) columns, and
// Graf's addition theorem (H_0(k|x-y|) = sum_l H_l(k|x|) e^{i l th_x}
// J_l(k|y|) e^{-i l th_y} for |x| > |y|) projects the monopole strengths onto
// the outgoing coefficients: alpha_l = sum_j c_j J_l(kp |y_j|) e^{-i l th_j}.
//
// Per particle the working matrix is [A | B], 2N rows and 2N + 2(2p+1)
// columns, column-major in HBM (2N <= 512: 4.7 MB at N = 256).  The LU
// factorisation with partial pivoting runs on the augmented matrix, so the
// row swaps and the elimination reach B as they happen (B becomes L^{-1} P B)
// and only the back substitution with U remains.  Blocked right-looking LU,
// panel width 16: a workgroup of 512 lanes owns one row per lane; the panel
// row lives in registers, the pivot row is broadcast through LDS, the U12
// block rows are solved one column per lane, and the trailing update streams
// each column once per panel (thread = row, coalesced).
#include "dev.h"
#include "ems_internal.h"

namespace ems {

namespace {

constexpr int kNB = 16;          // LU panel width
constexpr int kLuLanes = 512;    // one row of the working matrix per lane
constexpr int kRC = 31;          // right-hand sides per back-substitution pass (62 at p = 15)
constexpr int kCC = 192;         // trailing columns per LDS chunk of U12 (48 KB)
constexpr int kTG = 8;           // trailing columns per pipelined group
constexpr int kBB = 16;          // back-substitution rows per block (n2 is a multiple)
constexpr int kMaxJ = kMaxP + 3; // J_0 .. J_{p+2}

__device__ __forceinline__ double2 cinv(double2 d) {
  const double s = 1.0 / (d.x * d.x + d.y * d.y);
  return make_double2(d.x * s, -d.y * s);
}

// J_0..J_m (m < kMaxJ) and Y_0, Y_1 of a real x > 0 by Miller's backward
// recurrence J_{n-1} = (2n/x) J_n - J_{n+1}, normalised with
// J_0 + 2 sum_k J_{2k} = 1; Y_0 by the Neumann series
// Y_0 = (2/pi)[(ln(x/2) + gamma) J_0 - 2 sum_{k>=1} (-1)^k J_{2k}/k] and
// Y_1 = -Y_0' = (2/pi)[(ln(x/2) + gamma) J_1 - J_0/x
//               + sum_{k>=1} (-1)^k (J_{2k-1} - J_{2k+1})/k].
// Absolute accuracy a few 1e-15 for x up to 30 (and beyond: the start index
// grows with x).  m >= 1 (Y_1 uses J_1).
__device__ void bessel_jy(double x, int m, double *J, double &Y0, double &Y1) {
  const double xm = fmax(x, (double)m);
  const int n0 = 2 * ((int)(xm + 32.0) / 2);
  for (int n = 0; n <= m; ++n) J[n] = 0.0;
  double jp1 = 0.0, j = 1e-30, norm = 0.0, s0 = 0.0, s1 = 0.0;
  const double tx = 2.0 / x;
  for (int n = n0; n >= 1; --n) {
    const double jm1 = n * tx * j - jp1;
    if (n <= m) J[n] = j;
    if ((n & 1) == 0) {
      const int k = n >> 1;
      const double sg = (k & 1) ? -1.0 : 1.0;
      norm += 2.0 * j;
      s0 += sg * j / k;
      s1 += sg * (jm1 - jp1) / k;
    }
    jp1 = j;
    j = jm1;
    if (fabs(j) > 1e200) {
      j *= 1e-200;
      jp1 *= 1e-200;
      norm *= 1e-200;
      s0 *= 1e-200;
      s1 *= 1e-200;
      for (int q = 0; q <= m; ++q) J[q] *= 1e-200;
    }
  }
  norm += j;
  const double inv = 1.0 / norm;
  J[0] = j;
  for (int n = 0; n <= m; ++n) J[n] *= inv;
  s0 *= inv;
  s1 *= inv;
  const double L = log(0.5 * x) + 0.57721566490153286061;
  const double tp = 0.63661977236758134308;   // 2/pi
  Y0 = tp * (L * J[0] - 2.0 * s0);
  Y1 = tp * (L * J[1] - J[0] / x + s1);
}

// Point z(t + i delta) of shape kind (0 circle radius a, 1 ellipse semi-axes
// a and a/2, and the curves r = a (1 + eps cos(m t)): 2 star (m 5, eps 0.3),
// 3 pear (m 3, eps 1/4), 4 starfish (m 5, eps 1/4), the last two the paper's
// a1 + a2 cos(a3 t) with a2 = a1/4) turned by (ct, st) = e^{i theta0}, and
// dz/dt; complex numbers stand for points (Re, Im).
__device__ void shape_point(int kind, double a, double t, double delta, double ct, double st,
                            double2 &z, double2 &dz) {
  double s, c;
  sincos(t, &s, &c);
  const double ch = cosh(delta), sh = sinh(delta);
  const double2 cz = make_double2(c * ch, -s * sh);   // cos(t + i delta)
  const double2 sz = make_double2(s * ch, c * sh);    // sin(t + i delta)
  const double ed = exp(-delta);
  const double2 e = make_double2(c * ed, s * ed);     // e^{i (t + i delta)}
  if (kind == 0) {
    z = cscale(e, a);
    dz = make_double2(-z.y, z.x);
  } else if (kind == 1) {
    z = make_double2(a * cz.x - 0.5 * a * sz.y, a * cz.y + 0.5 * a * sz.x);
    dz = make_double2(-a * sz.x - 0.5 * a * cz.y, -a * sz.y + 0.5 * a * cz.x);
  } else {
    const double m = kind == 3 ? 3.0 : 5.0, eps = kind == 2 ? 0.3 : 0.25;
    double s5, c5;
    sincos(m * t, &s5, &c5);
    const double ch5 = cosh(m * delta), sh5 = sinh(m * delta);
    const double2 c5z = make_double2(c5 * ch5, -s5 * sh5);   // cos(m (t + i delta))
    const double2 s5z = make_double2(s5 * ch5, c5 * sh5);    // sin(m (t + i delta))
    const double2 r = make_double2(a * (1.0 + eps * c5z.x), a * eps * c5z.y);
    const double2 dr = cscale(s5z, -eps * m * a);
    z = cmul(r, e);
    dz = cmul(make_double2(dr.x - r.y, dr.y + r.x), e);
  }
  const double2 rot = make_double2(ct, st);
  z = cmul(z, rot);
  dz = cmul(dz, rot);
}

struct ShapeArgs {
  const int *kind;
  const double *a, *ct, *st, *delta;
  const int *p, *bc;
};

__device__ __forceinline__ void collocation(const ShapeArgs &g, int m, int i, int N, double2 &z,
                                            double &nx, double &ny) {
  double2 dz;
  shape_point(g.kind[m], g.a[m], 6.283185307179586477 * i / N, 0.0, g.ct[m], g.st[m], z, dz);
  const double ad = 1.0 / hypot(dz.x, dz.y);
  nx = dz.y * ad;
  ny = -dz.x * ad;
}

__device__ __forceinline__ double2 source(const ShapeArgs &g, int m, int j, int N) {
  double2 z, dz;
  shape_point(g.kind[m], g.a[m], 6.283185307179586477 * j / N, g.delta[m], g.ct[m], g.st[m], z,
              dz);
  return z;
}

// Collocation matrix A: thread per (collocation point i, source j), H_0 and
// H_1 from the device library's Bessel functions of order 0 and 1; rows
// comp * N + i (comp 0, 1 of u or sigma.nu), columns w * N + j (w 0: the
// compressional monopole, w 1: the shear one).  For f = H_0(k rho) about the
// source, grad f = -k H_1 e and Hess f = -k^2 H_0 e e^T + (k H_1 / rho)(2 e e^T - I),
// e the unit vector from the source.
__global__ __launch_bounds__(256) void mfs_matrix_kernel(ShapeArgs g, int i0, int N,
                                                          int64_t mstride, double kp, double ks,
                                                          double lam, double mu,
                                                          double2 *__restrict__ W) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= N * N) return;
  const int mloc = blockIdx.y, m = i0 + mloc;
  const int i = idx % N, j = idx / N;
  const int n2 = 2 * N;
  double2 zc;
  double nx, ny;
  collocation(g, m, i, N, zc, nx, ny);
  const double2 zs = source(g, m, j, N);
  const double dx = zc.x - zs.x, dy = zc.y - zs.y;
  const double rho = hypot(dx, dy);
  const double ex = dx / rho, ey = dy / rho;
  const int bc = g.bc[m];
  double2 *Wm = W + (int64_t)mloc * mstride;
  for (int w = 0; w < 2; ++w) {
    const double k = w == 0 ? kp : ks;
    const double z = k * rho;
    const double2 H0 = make_double2(j0(z), y0(z)), H1 = make_double2(j1(z), y1(z));
    const double2 gx = cscale(H1, -k * ex), gy = cscale(H1, -k * ey);
    const double2 c1 = cscale(H0, -k * k), c2 = cscale(H1, k / rho);
    const double2 hxx = cadd(cscale(c1, ex * ex), cscale(c2, 2.0 * ex * ex - 1.0));
    const double2 hxy = cadd(cscale(c1, ex * ey), cscale(c2, 2.0 * ex * ey));
    const double2 hyy = cadd(cscale(c1, ey * ey), cscale(c2, 2.0 * ey * ey - 1.0));
    double2 v0, v1;
    if (bc == 0) {
      if (w == 0) {
        v0 = gx;
        v1 = gy;
      } else {
        v0 = cscale(gy, -1.0);
        v1 = gx;
      }
    } else {
      double2 s11, s22, s12;
      if (w == 0) {
        const double2 lap = cadd(hxx, hyy);
        s11 = cadd(cscale(lap, lam), cscale(hxx, 2.0 * mu));
        s22 = cadd(cscale(lap, lam), cscale(hyy, 2.0 * mu));
        s12 = cscale(hxy, 2.0 * mu);
      } else {
        s11 = cscale(hxy, -2.0 * mu);
        s22 = cscale(hxy, 2.0 * mu);
        s12 = cscale(csub(hxx, hyy), mu);
      }
      v0 = cadd(cscale(s11, nx), cscale(s12, ny));
      v1 = cadd(cscale(s12, nx), cscale(s22, ny));
    }
    double2 *col = Wm + (int64_t)(w * N + j) * n2;
    col[i] = v0;
    col[N + i] = v1;
  }
}

// Incident columns B (minus the incident displacement or traction of each
// basis field), thread per collocation point; v_n = J_n(k r) e^{i n th} and
// its derivatives by d_x v_n = (k/2)(v_{n-1} - v_{n+1}),
// d_y v_n = (i k/2)(v_{n-1} + v_{n+1}), applied twice.
__global__ __launch_bounds__(128) void mfs_rhs_kernel(ShapeArgs g, int i0, int N, int64_t mstride,
                                                      double kp, double ks, double lam, double mu,
                                                      double2 *__restrict__ W) {
  const int i = blockIdx.x * 128 + threadIdx.x;
  if (i >= N) return;
  const int mloc = blockIdx.y, m = i0 + mloc;
  const int n2 = 2 * N, pm = g.p[m], Nm = 2 * pm + 1, bc = g.bc[m];
  double2 zc;
  double nx, ny;
  collocation(g, m, i, N, zc, nx, ny);
  const double r = hypot(zc.x, zc.y);
  const double2 eth = make_double2(zc.x / r, zc.y / r);
  double2 ep[kMaxJ];   // e^{i q th}, q = 0..p+2
  ep[0] = make_double2(1.0, 0.0);
  for (int q = 1; q <= pm + 2; ++q) ep[q] = cmul(ep[q - 1], eth);
  double2 *Wm = W + (int64_t)mloc * mstride;
  for (int w = 0; w < 2; ++w) {
    const double k = w == 0 ? kp : ks;
    double J[kMaxJ], Y0, Y1;
    bessel_jy(k * r, pm + 2, J, Y0, Y1);
    auto v = [&](int q) -> double2 {
      const int aq = q < 0 ? -q : q;
      double jv = J[aq];
      double2 e = ep[aq];
      if (q < 0) {
        if (aq & 1) jv = -jv;
        e.y = -e.y;
      }
      return cscale(e, jv);
    };
    const double h = 0.5 * k, h2 = 0.25 * k * k;
    for (int n = -pm; n <= pm; ++n) {
      const double2 vm2 = v(n - 2), vm1 = v(n - 1), v0 = v(n), vp1 = v(n + 1), vp2 = v(n + 2);
      const double2 vx = cscale(csub(vm1, vp1), h);
      const double2 sy = cscale(cadd(vm1, vp1), h);
      const double2 vy = make_double2(-sy.y, sy.x);
      const double2 vxx = cscale(cadd(csub(vm2, cscale(v0, 2.0)), vp2), h2);
      const double2 txy = cscale(csub(vm2, vp2), h2);
      const double2 vxy = make_double2(-txy.y, txy.x);
      const double2 vyy = cscale(cadd(cadd(vm2, cscale(v0, 2.0)), vp2), -h2);
      double2 c0, c1;
      if (bc == 0) {
        if (w == 0) {
          c0 = vx;
          c1 = vy;
        } else {
          c0 = cscale(vy, -1.0);
          c1 = vx;
        }
      } else {
        double2 s11, s22, s12;
        if (w == 0) {
          const double2 lap = cadd(vxx, vyy);
          s11 = cadd(cscale(lap, lam), cscale(vxx, 2.0 * mu));
          s22 = cadd(cscale(lap, lam), cscale(vyy, 2.0 * mu));
          s12 = cscale(vxy, 2.0 * mu);
        } else {
          s11 = cscale(vxy, -2.0 * mu);
          s22 = cscale(vxy, 2.0 * mu);
          s12 = cscale(csub(vxx, vyy), mu);
        }
        c0 = cadd(cscale(s11, nx), cscale(s12, ny));
        c1 = cadd(cscale(s12, nx), cscale(s22, ny));
      }
      double2 *col = Wm + (int64_t)(n2 + w * Nm + n + pm) * n2;
      col[i] = cscale(c0, -1.0);
      col[N + i] = cscale(c1, -1.0);
    }
  }
}

// Blocked LU with partial pivoting (pivot = largest |Re| + |Im|, ties to the
// lower row index) of [A | B], one workgroup of 512 lanes per matrix, lane
// r = row r.  The L factor's columns left of the panel are never read again
// (B already carries L^{-1} P), so row swaps are applied to the columns right
// of the panel only.  info[m] is set when a pivot is exactly zero.  B has
// fixed_rhs columns, or 2 (2 p + 1) (the particle's incident basis) when
// fixed_rhs is 0.
__global__ __launch_bounds__(kLuLanes) void mfs_lu_kernel(double2 *__restrict__ W, int n2,
                                                         int64_t mstride,
                                                         const int *__restrict__ p, int i0,
                                                         int *__restrict__ info, int fixed_rhs) {
  __shared__ double2 urow[kNB], krow[kNB];
  __shared__ double2 L11[kNB][kNB];
  __shared__ double2 Us[kCC][kNB];
  __shared__ int ipiv[kNB];
  __shared__ int prow[2 * kNB], psrc[2 * kNB];   // net row permutation of a panel
  __shared__ int pcnt;
  __shared__ double redv[kLuLanes / 64];
  __shared__ int redi[kLuLanes / 64];
  const int mloc = blockIdx.x;
  double2 *A = W + (int64_t)mloc * mstride;
  const int ncol = n2 + (fixed_rhs > 0 ? fixed_rhs : 2 * (2 * p[i0 + mloc] + 1));
  const int r = threadIdx.x, lane = r & 63, wv = r >> 6;
  for (int k0 = 0; k0 < n2; k0 += kNB) {
    double2 pr[kNB];
    const bool mine = r >= k0 && r < n2;
#pragma unroll
    for (int jj = 0; jj < kNB; ++jj)
      pr[jj] = mine ? A[(int64_t)(k0 + jj) * n2 + r] : make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < kNB; ++j) {
      const int kk = k0 + j;
      double v = (r >= kk && r < n2) ? fabs(pr[j].x) + fabs(pr[j].y) : -1.0;
      int id = r;
      for (int o = 32; o > 0; o >>= 1) {
        const double v2 = __shfl_xor(v, o);
        const int i2 = __shfl_xor(id, o);
        if (v2 > v || (v2 == v && i2 < id)) {
          v = v2;
          id = i2;
        }
      }
      if (lane == 0) {
        redv[wv] = v;
        redi[wv] = id;
      }
      __syncthreads();
      v = redv[0];
      id = redi[0];
      for (int q = 1; q < kLuLanes / 64; ++q) {
        const double v2 = redv[q];
        const int i2 = redi[q];
        if (v2 > v || (v2 == v && i2 < id)) {
          v = v2;
          id = i2;
        }
      }
      const int pv = id;
      if (r == pv) {
#pragma unroll
        for (int jj = 0; jj < kNB; ++jj) urow[jj] = pr[jj];
      }
      if (r == kk && pv != kk) {
#pragma unroll
        for (int jj = 0; jj < kNB; ++jj) krow[jj] = pr[jj];
      }
      if (r == 0) {
        ipiv[j] = pv;
        if (!(v > 0.0)) info[mloc] = 1;
      }
      __syncthreads();
      if (pv != kk) {
        if (r == kk) {
#pragma unroll
          for (int jj = 0; jj < kNB; ++jj) pr[jj] = urow[jj];
        } else if (r == pv) {
#pragma unroll
          for (int jj = 0; jj < kNB; ++jj) pr[jj] = krow[jj];
        }
      }
      if (r > kk && r < n2 && v > 0.0) {
        const double2 l = cmul(pr[j], cinv(urow[j]));
        pr[j] = l;
#pragma unroll
        for (int jj = j + 1; jj < kNB; ++jj) pr[jj] = csub(pr[jj], cmul(l, urow[jj]));
      }
      // the next step's writes of redv/urow/krow come after its first barrier,
      // which every lane reaches only after its reads of this step
    }
    if (mine) {
#pragma unroll
      for (int jj = 0; jj < kNB; ++jj) A[(int64_t)(k0 + jj) * n2 + r] = pr[jj];
    }
    if (r >= k0 && r < k0 + kNB) {
#pragma unroll
      for (int jj = 0; jj < kNB; ++jj) L11[r - k0][jj] = pr[jj];
    }
    if (r == 0) {
      // the panel's swaps (k0 + j <-> ipiv[j], in order) as one permutation of
      // at most 2 kNB rows: after them row prow[i] holds the old row psrc[i];
      // entries 0..kNB-1 are the panel rows themselves
      int cnt = kNB;
      for (int j = 0; j < kNB; ++j) prow[j] = psrc[j] = k0 + j;
      for (int j = 0; j < kNB; ++j) {
        const int pv = ipiv[j];
        int b = -1;
        if (pv < k0 + kNB) {
          b = pv - k0;
        } else {
          for (int i = kNB; i < cnt; ++i)
            if (prow[i] == pv) b = i;
          if (b < 0) {
            prow[cnt] = psrc[cnt] = pv;
            b = cnt++;
          }
        }
        const int tmp = psrc[j];
        psrc[j] = psrc[b];
        psrc[b] = tmp;
      }
      pcnt = cnt;
    }
    __syncthreads();
    const int c1 = k0 + kNB;
    // columns right of the panel in chunks of kCC: row swaps and
    // U12 = L11^{-1} A12 (lane per column, kept in LDS), then the trailing
    // update A22 -= L21 U12 (lane per row, software-pipelined column groups)
    for (int cb = c1; cb < ncol; cb += kCC) {
      const int cn = min(kCC, ncol - cb);
      if (r < cn) {
        // keeps the L11 reads inside the chunk loop (hoisted, 120 complex
        // values would not fit in registers)
        asm volatile("" ::: "memory");
        double2 *col = A + (int64_t)(cb + r) * n2;
        // every load of the permutation first (independent), then the stores
        const int cnt = pcnt;
        double2 u[kNB], ext[kNB];
#pragma unroll
        for (int jj = 0; jj < kNB; ++jj) u[jj] = col[psrc[jj]];
#pragma unroll
        for (int i = 0; i < kNB; ++i)
          ext[i] = kNB + i < cnt ? col[psrc[kNB + i]] : make_double2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < kNB; ++i)
          if (kNB + i < cnt) col[prow[kNB + i]] = ext[i];
#pragma unroll
        for (int jj = 1; jj < kNB; ++jj)
#pragma unroll
          for (int ii = 0; ii < jj; ++ii) u[jj] = csub(u[jj], cmul(L11[jj][ii], u[ii]));
#pragma unroll
        for (int jj = 0; jj < kNB; ++jj) {
          col[k0 + jj] = u[jj];
          Us[r][jj] = u[jj];
        }
      }
      __syncthreads();
      if (r >= c1 && r < n2) {
        // groups of kTG columns, the next group's loads in flight while the
        // current one is updated
        double2 cur[kTG], nxt[kTG];
#pragma unroll
        for (int u = 0; u < kTG; ++u)
          cur[u] = u < cn ? A[(int64_t)(cb + u) * n2 + r] : make_double2(0.0, 0.0);
        for (int q = 0; q < cn; q += kTG) {
          if (q + kTG < cn) {
#pragma unroll
            for (int u = 0; u < kTG; ++u)
              nxt[u] = q + kTG + u < cn ? A[(int64_t)(cb + q + kTG + u) * n2 + r]
                                        : make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int u = 0; u < kTG; ++u) {
            if (q + u < cn) {
              double2 a0 = cur[u];
#pragma unroll
              for (int jj = 0; jj < kNB; ++jj) a0 = csub(a0, cmul(pr[jj], Us[q + u][jj]));
              A[(int64_t)(cb + q + u) * n2 + r] = a0;
            }
          }
#pragma unroll
          for (int u = 0; u < kTG; ++u) cur[u] = nxt[u];
        }
      }
      __syncthreads();
    }
  }
}

// Back substitution U X = Y on the right-hand-side columns, in place, by
// blocks of kBB rows from the bottom: lane r holds row r of kRC columns in
// registers; the rows of a block stage their values and the block's diagonal
// U in LDS, lane q < kRC solves the small triangular system for column q,
// and every row above subtracts the block's contribution (kBB independent
// loads of its U entries).  Three barriers per block instead of one per row.
__global__ __launch_bounds__(kLuLanes) void mfs_backsolve_kernel(double2 *__restrict__ W, int n2,
                                                                int64_t mstride,
                                                                const int *__restrict__ p,
                                                                int i0, int fixed_rhs) {
  __shared__ double2 Ub[kBB][kBB];
  __shared__ double2 yb[kBB][kRC];
  const int mloc = blockIdx.x;
  double2 *A = W + (int64_t)mloc * mstride;
  const int nr = fixed_rhs > 0 ? fixed_rhs : 2 * (2 * p[i0 + mloc] + 1);
  const int r = threadIdx.x;
  for (int c0 = 0; c0 < nr; c0 += kRC) {
    const int nc = min(kRC, nr - c0);
    double2 y[kRC];
#pragma unroll
    for (int q = 0; q < kRC; ++q)
      y[q] = (r < n2 && q < nc) ? A[(int64_t)(n2 + c0 + q) * n2 + r] : make_double2(0.0, 0.0);
    for (int k0 = n2 - kBB; k0 >= 0; k0 -= kBB) {   // n2 is a multiple of kBB
      const bool blk = r >= k0 && r < k0 + kBB;
      if (blk) {
#pragma unroll
        for (int q = 0; q < kRC; ++q) yb[r - k0][q] = y[q];
      }
      if (r < kBB * kBB) {
        const int i = r % kBB, j = r / kBB;
        Ub[i][j] = A[(int64_t)(k0 + j) * n2 + k0 + i];
      }
      __syncthreads();
      if (r < nc) {
        for (int i = kBB - 1; i >= 0; --i) {
          double2 s = yb[i][r];
          for (int j = i + 1; j < kBB; ++j) s = csub(s, cmul(Ub[i][j], yb[j][r]));
          yb[i][r] = cmul(s, cinv(Ub[i][i]));
        }
      }
      __syncthreads();
      if (blk) {
#pragma unroll
        for (int q = 0; q < kRC; ++q) y[q] = yb[r - k0][q];
      } else if (r < k0) {
        double2 u[kBB];
#pragma unroll
        for (int j = 0; j < kBB; ++j) u[j] = A[(int64_t)(k0 + j) * n2 + r];
#pragma unroll
        for (int j = 0; j < kBB; ++j)
#pragma unroll
          for (int q = 0; q < kRC; ++q) y[q] = csub(y[q], cmul(u[j], yb[j][q]));
      }
      __syncthreads();
    }
    if (r < n2) {
#pragma unroll
      for (int q = 0; q < kRC; ++q)
        if (q < nc) A[(int64_t)(n2 + c0 + q) * n2 + r] = y[q];
    }
  }
}

// Projection table E[w][l][j] = J_{n}(k_w |y_j|) e^{-i n th_j}, n = l - p, thread
// per source.
__global__ __launch_bounds__(128) void mfs_proj_table_kernel(ShapeArgs g, int i0, int N,
                                                             int64_t estride, double kp,
                                                             double ks,
                                                             double2 *__restrict__ E) {
  const int j = blockIdx.x * 128 + threadIdx.x;
  if (j >= N) return;
  const int mloc = blockIdx.y, m = i0 + mloc;
  const int pm = g.p[m], Nm = 2 * pm + 1;
  const double2 zs = source(g, m, j, N);
  const double r = hypot(zs.x, zs.y);
  const double2 emth = make_double2(zs.x / r, -zs.y / r);   // e^{-i th}
  double2 *Em = E + (int64_t)mloc * estride;
  for (int w = 0; w < 2; ++w) {
    double J[kMaxJ], Y0, Y1;
    bessel_jy((w == 0 ? kp : ks) * r, pm < 1 ? 1 : pm, J, Y0, Y1);
    double2 e = make_double2(1.0, 0.0);
    for (int q = 0; q <= pm; ++q) {
      // n = q: J_q e^{-i q th}; n = -q: (-1)^q J_q e^{+i q th}
      const double2 pos = cscale(e, J[q]);
      const double2 neg = cscale(make_double2(e.x, -e.y), (q & 1) ? -J[q] : J[q]);
      Em[((int64_t)w * Nm + pm + q) * N + j] = pos;
      Em[((int64_t)w * Nm + pm - q) * N + j] = neg;
      e = cmul(e, emth);
    }
  }
}

// S[row][col] = sum_j E[w][l][j] X[w N + j][col], row = w (2p+1) + l; thread per
// entry, written row-major into the packed output.
__global__ __launch_bounds__(256) void mfs_project_kernel(const double2 *__restrict__ W,
                                                          const double2 *__restrict__ E, int N,
                                                          int64_t mstride, int64_t estride,
                                                          const int *__restrict__ p,
                                                          const int64_t *__restrict__ Soff,
                                                          int i0, double2 *__restrict__ S) {
  const int mloc = blockIdx.y, m = i0 + mloc;
  const int pm = p[m], Nm = 2 * pm + 1, nr = 2 * Nm;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nr * nr) return;
  const int row = idx / nr, col = idx % nr;
  const int w = row / Nm, l = row % Nm;
  const int n2 = 2 * N;
  const double2 *x = W + (int64_t)mloc * mstride + (int64_t)(n2 + col) * n2 + w * N;
  const double2 *e = E + (int64_t)mloc * estride + ((int64_t)w * Nm + l) * N;
  double2 s = make_double2(0.0, 0.0);
  for (int j = 0; j < N; ++j) cfma(s, e[j], x[j]);
  S[Soff[m] + idx] = s;
}

}  // namespace

hipError_t launch_lu_solve_batch(double2 *W, int n2, int64_t mstride, int cnt, int nrhs,
                                 int *info, hipStream_t st) {
  if (n2 > kLuLanes || n2 % kNB != 0 || n2 % kBB != 0 || nrhs <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mfs_lu_kernel, dim3(cnt), dim3(kLuLanes), 0, st, W, n2, mstride, nullptr, 0,
                     info, nrhs);
  hipLaunchKernelGGL(mfs_backsolve_kernel, dim3(cnt), dim3(kLuLanes), 0, st, W, n2, mstride,
                     nullptr, 0, nrhs);
  return hipGetLastError();
}

hipError_t launch_mfs_smatrices(const MfsBatch &b, int i0, int cnt, double2 *W, int64_t mstride,
                                double2 *E, int64_t estride, int *info, double2 *S,
                                hipStream_t st) {
  const ShapeArgs g{b.kind, b.a, b.ct, b.st, b.delta, b.p, b.bc};
  const int N = b.npts, n2 = 2 * N;
  if (n2 > kLuLanes || n2 % kNB != 0) return hipErrorInvalidValue;
  const double kp = b.md->kp, ks = b.md->ks, lam = b.md->lam_h, mu = b.md->mu_h;
  hipLaunchKernelGGL(mfs_matrix_kernel, dim3((N * N + 255) / 256, cnt), dim3(256), 0, st, g, i0,
                     N, mstride, kp, ks, lam, mu, W);
  hipLaunchKernelGGL(mfs_rhs_kernel, dim3((N + 127) / 128, cnt), dim3(128), 0, st, g, i0, N,
                     mstride, kp, ks, lam, mu, W);
  hipLaunchKernelGGL(mfs_proj_table_kernel, dim3((N + 127) / 128, cnt), dim3(128), 0, st, g, i0,
                     N, estride, kp, ks, E);
  hipLaunchKernelGGL(mfs_lu_kernel, dim3(cnt), dim3(kLuLanes), 0, st, W, n2, mstride, b.p, i0,
                     info, 0);
  hipLaunchKernelGGL(mfs_backsolve_kernel, dim3(cnt), dim3(kLuLanes), 0, st, W, n2, mstride, b.p,
                     i0, 0);
  const int nrmax = 2 * (2 * kMaxP + 1);
  hipLaunchKernelGGL(mfs_project_kernel, dim3((nrmax * nrmax + 255) / 256, cnt), dim3(256), 0, st,
                     W, E, N, mstride, estride, b.p, b.Soff, i0, S);
  return hipGetLastError();
}

}  // namespace ems
