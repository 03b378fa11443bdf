// Host set-up of the operator: wavenumbers, Sommerfeld node tables, the
// per-node welded-interface reflection, closed-form disk scattering matrices.
#include <algorithm>
#include <cmath>
#include <cstdio>

#include "ems_internal.h"

namespace ems {

static const double kPi = 3.14159265358979323846;

Media make_media(const ems_media &m) {
  Media d{};
  d.lam_h = m.host.lambda;
  d.mu_h = m.host.mu;
  d.rho_h = m.host.rho;
  d.lam_b = m.substrate.lambda;
  d.mu_b = m.substrate.mu;
  d.rho_b = m.substrate.rho;
  d.omega = m.omega;
  // Helmholtz split (Section 2) with the density kept.
  d.kp = m.omega * std::sqrt(d.rho_h / (d.lam_h + 2.0 * d.mu_h));
  d.ks = m.omega * std::sqrt(d.rho_h / d.mu_h);
  d.kpb = m.omega * std::sqrt(d.rho_b / (d.lam_b + 2.0 * d.mu_b));
  d.ksb = m.omega * std::sqrt(d.rho_b / d.mu_b);
  return d;
}

cd branch_s(cd xi, double k) {
  if (xi.imag() == 0.0) {
    const double x = xi.real();
    const double v = (x - k) * (x + k);
    if (v > 0) return cd(std::sqrt(v), 0.0);
    return cd(0.0, -std::sqrt(-v));
  }
  return cd(0.0, -1.0) * std::sqrt(cd(k * k, 0.0) - xi * xi);
}

// ---------------------------------------------------------------------------
// Gauss-Legendre rule on [-1, 1] by Newton iteration on P_n.
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 0; j < n; ++j) {
        const double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j + 1.0) * z * p2 - j * p3) / (j + 1.0);
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      const double z1 = z;
      z = z1 - p1 / pp;
      if (std::fabs(z - z1) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

// Decay bound of the Sommerfeld integrand tail: exp(-t D) (2t/k + 1)^(2p)
// for the depth sum D of a pair; its logarithm peaks at some t.
static double bound_peak(double dmin, int pmax, double kmin) {
  double peak = -1e300;
  for (double t = 0.0; t < 4000.0; t += 0.01)
    peak = std::max(peak, -t * dmin + 2.0 * pmax * std::log(2.0 * t / kmin + 1.0));
  return peak;
}

static double auto_tmax(double dmin, int pmax, double kmin, double kmax) {
  const double peak = bound_peak(dmin, pmax, kmin);
  for (double t = kmax + 2.0; t < 4000.0; t += 0.01) {
    const double v = -t * dmin + 2.0 * pmax * std::log(2.0 * t / kmin + 1.0);
    if (v < peak + std::log(1e-18)) return t;
  }
  return 4000.0;
}

namespace {
struct PanelRule {
  std::vector<double> gx, gw;   // bulk rule
  int n = 0;
};

void push(NodeTable &out, cd xi, cd w, double bp, double d) {
  out.xi.push_back(xi);
  out.w.push_back(w);
  out.bp.push_back(bp);
  out.d.push_back(d);
}

void add_panel(const PanelRule &r, double a, double b, NodeTable &out) {
  const double c = 0.5 * (a + b), hl = 0.5 * (b - a);
  for (int i = 0; i < r.n; ++i) push(out, cd(c + hl * r.gx[i], 0.0), cd(hl * r.gw[i], 0.0), 0.0, 0.0);
}

// Panel next to a branch point at `bp`, extending by `len` towards `dir`
// (+1 right, -1 left): xi = bp + dir u^2, u in [0, sqrt(len)].
void add_sub_panel(const PanelRule &r, double bp, double len, int dir, NodeTable &out) {
  const double U = std::sqrt(len), c = 0.5 * U, hl = 0.5 * U;
  for (int i = 0; i < r.n; ++i) {
    const double u = c + hl * r.gx[i];
    push(out, cd(bp + dir * u * u, 0.0), cd(hl * r.gw[i] * 2.0 * u, 0.0), bp, dir * u * u);
  }
}

// Half interval from a singular end `bp` towards `mid` (dir = sign(mid - bp)):
// substitution panel, geometrically graded panels, then uniform panels.
void graded_half(const PanelRule &r, double bp, double mid, double Lb, double Losc,
                 NodeTable &out) {
  const int dir = mid > bp ? 1 : -1;
  const double span = std::fabs(mid - bp);
  double Lsub = std::min(Lb, 0.5 * span);
  add_sub_panel(r, bp, Lsub, dir, out);
  double pos = Lsub, len = Lsub;
  while (pos < span) {
    double nl = std::min(2.0 * len, Losc);
    if (nl >= Losc) break;
    if (pos + nl > span) break;
    add_panel(r, std::min(bp + dir * pos, bp + dir * (pos + nl)),
              std::max(bp + dir * pos, bp + dir * (pos + nl)), out);
    pos += nl;
    len = nl;
  }
  const double rest = span - pos;
  if (rest > 1e-15) {
    const int np = std::max(1, (int)std::ceil(rest / Losc - 1e-9));
    const double h = rest / np;
    for (int i = 0; i < np; ++i) {
      const double a = bp + dir * (pos + i * h), b = bp + dir * (pos + (i + 1) * h);
      add_panel(r, std::min(a, b), std::max(a, b), out);
    }
  }
}
}  // namespace

int build_nodes(const SommerfeldSpec &spec, const Media &md, const std::vector<double> &xy,
                const std::vector<int> &p, NodeTable &out, std::string &err) {
  out.xi.clear();
  out.w.clear();
  out.bp.clear();
  out.d.clear();
  const int n = (int)p.size();
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  int pmax = 0;
  for (int i = 0; i < n; ++i) {
    xmin = std::min(xmin, xy[2 * i]);
    xmax = std::max(xmax, xy[2 * i]);
    ymin = std::min(ymin, -xy[2 * i + 1]);
    ymax = std::max(ymax, -xy[2 * i + 1]);
    pmax = std::max(pmax, p[i]);
  }
  const double X = std::max(xmax - xmin, 1e-3);
  const double Dmin = 2.0 * ymin, Dmax = 2.0 * ymax;
  const double kmin = std::min(md.kp, md.ks);
  const double kmax = std::max(std::max(md.kp, md.ks), std::max(md.kpb, md.ksb));
  double T = spec.t_max > 0 ? spec.t_max : auto_tmax(Dmin, pmax, kmin, kmax);
  out.t_max = T;
  if (spec.kind == 2) {
    if ((int)spec.user.size() != 4 * spec.q || spec.q <= 0) {
      err = "sommerfeld kind 2 needs q > 0 user nodes";
      return EMS_ERR_ARG;
    }
    for (int j = 0; j < spec.q; ++j)
      push(out, cd(spec.user[4 * j], spec.user[4 * j + 1]),
           cd(spec.user[4 * j + 2], spec.user[4 * j + 3]), 0.0, 0.0);
    return EMS_OK;
  }
  if (spec.kind == 0) {
    // Section 5.1: xi(t) = t - i delta tanh(t), trapezoidal rule in t.
    const int q = spec.q > 1 ? spec.q : 512;
    const double h = 2.0 * T / (q - 1);
    for (int j = 0; j < q; ++j) {
      const double t = -T + j * h;
      const double th = std::tanh(t);
      const double sech2 = 1.0 - th * th;
      const double wt = (j == 0 || j == q - 1) ? 0.5 * h : h;
      push(out, cd(t, -spec.delta * th), wt * cd(1.0, -spec.delta * sech2), 0.0, 0.0);
    }
    return EMS_OK;
  }
  if (spec.kind != 1 && spec.kind != 3) {
    err = "unknown sommerfeld kind";
    return EMS_ERR_ARG;
  }
  // Real axis.  Core |xi| <= K + b around the branch points: composite
  // Gauss-Legendre panels, graded towards every branch point with a
  // xi = k +- u^2 panel next to it.  With spec.kind == 1 the tails
  // |xi| >= K use the trapezoidal rule on a smooth partition of unity:
  // chi = 1 on |xi| <= K, chi = erfc(beta (2t - 1)) / 2 for t = (|xi| - K)/b
  // in [0, 1], 0 beyond.  The core panels carry chi, the tail nodes 1 - chi;
  // f (1 - chi) is smooth and vanishes at |xi| = K, so the trapezoidal rule
  // is spectrally accurate there once 2 pi / h exceeds the horizontal
  // spread X plus the width of the window's and f's spectra.  kind 3 keeps
  // Gauss-Legendre panels everywhere.
  PanelRule r;
  r.n = spec.panel_order;
  gauss_legendre(r.n, r.gx, r.gw);
  // A panel of n Gauss points is exact to degree 2n - 1.  The integrand is a
  // plane wave of frequency sqrt(X^2 + D^2) (horizontal spread X, depth sum
  // D) times powers zeta^(n + n') of degree up to 2 p_max.  Measured against
  // the multipole-to-Sommerfeld lemma at orders +-2p and against the
  // oracle at the 20000-particle cloud, (half-length) x (frequency) must
  // stay below about 1.2 n - 2 p_max - 8.
  const double wmax = std::max(8.0, 1.2 * r.n - 2.0 * pmax - 8.0);
  const double freq = std::sqrt(X * X + Dmax * Dmax);
  double Losc = std::min(2.0, 2.0 * wmax / freq) * spec.panel_scale;
  std::vector<double> bps = {md.kp, md.ks, md.kpb, md.ksb};
  std::sort(bps.begin(), bps.end());
  bps.erase(std::unique(bps.begin(), bps.end(),
                        [](double a, double b) { return std::fabs(a - b) < 1e-12; }),
            bps.end());
  std::vector<double> pts;
  for (auto it = bps.rbegin(); it != bps.rend(); ++it) pts.push_back(-*it);
  for (double b : bps) pts.push_back(b);
  const bool hybrid = spec.kind == 1;
  const double a_margin = 1.5, b_win = 2.5, beta = 6.0;
  const double K = pts.back() + a_margin;
  const double core_end = hybrid ? K + b_win : T;
  if (T <= core_end + 0.5) T = core_end + 0.5;
  out.t_max = T;
  // Substitution panel [bp, bp + L] in u = sqrt(|xi - bp|): the chirp
  // e^{i X u^2} gives u-frequency 2 X u and the depth factor e^{-sqrt(2k) u D}
  // a rate sqrt(2k) D; over half the u-interval sqrt(L)/2 the combined
  // (X L)^2 + (k L / 2) D^2 must stay below wsub^2.
  const double wsub = 18.0;
  auto Lb_of = [&](double b) {
    const double kb = std::max(std::fabs(b), 1e-3);
    const double bq = 0.5 * kb * Dmax * Dmax;
    const double L = (-bq + std::sqrt(bq * bq + 4.0 * X * X * wsub * wsub)) / (2.0 * X * X);
    return std::min(0.5 * Losc, L);
  };
  graded_half(r, pts.front(), -core_end, Lb_of(pts.front()), Losc, out);
  for (size_t i = 0; i + 1 < pts.size(); ++i) {
    const double a = pts[i], b = pts[i + 1], mid = 0.5 * (a + b);
    graded_half(r, a, mid, Lb_of(a), Losc, out);
    graded_half(r, b, mid, Lb_of(b), Losc, out);
  }
  graded_half(r, pts.back(), core_end, Lb_of(pts.back()), Losc, out);
  if (hybrid) {
    auto chi = [&](double x) {
      const double t = (std::fabs(x) - K) / b_win;
      if (t <= 0) return 1.0;
      if (t >= 1) return 0.0;
      return 0.5 * std::erfc(beta * (2.0 * t - 1.0));
    };
    for (size_t j = 0; j < out.xi.size(); ++j) out.w[j] *= chi(out.xi[j].real());
    // tail step: 2 pi / h >= tail_factor (X + 16 beta / b + 40)
    const double nu = spec.tail_factor * (X + 16.0 * beta / b_win + 40.0);
    const double h = 2.0 * kPi / nu;
    for (int side = -1; side <= 1; side += 2)
      for (int j = 1;; ++j) {
        const double x = K + j * h;
        if (x > T) break;
        const double wgt = h * (1.0 - chi(x));
        push(out, cd(side * x, 0.0), cd(wgt, 0.0), 0.0, 0.0);
      }
  }
  // sort by xi (helps locality; the sum is order independent up to rounding)
  std::vector<size_t> idx(out.xi.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(),
            [&](size_t a, size_t b) { return out.xi[a].real() < out.xi[b].real(); });
  NodeTable s;
  s.t_max = out.t_max;
  for (size_t i : idx) push(s, out.xi[i], out.w[i], out.bp[i], out.d[i]);
  out = s;
  return EMS_OK;
}

// Depth truncation.  The term that particle m sends through node xi_j (wave
// w) to particle l carries exp(-Re s_w(xi_j) d_m) on the source side and
// exp(-Re s_w'(xi_j) d_l) on the receiving side (d = depth below the
// interface), times powers of zeta of order up to p on each side, each at
// most (2|xi|/k_min + 1)^p in modulus on the real axis.  This is the tail
// bound by which t_max is placed (one factor per end of the pair, with s in
// place of |xi|).  A (node, particle) pair is left out of both contractions
// when its bound, with the shallowest particle at the other end, is below
// eps times the peak of that bound for the shallowest pair.  The bound falls
// with depth, so each node keeps a prefix of the particles in depth order,
// and the other end may be taken shallower (receivers above the particles);
// and each particle a set of nodes whose hull is recorded.  Complex nodes
// (the tanh contour, user nodes off the axis) keep every particle.
void depth_cuts(const NodeTable &nodes, const Media &md, const std::vector<double> &xy, int pmax,
                double eps, double dother, DepthCuts &out) {
  const int n = (int)(xy.size() / 2), q = (int)nodes.xi.size();
  std::vector<double> depth(n);
  for (int i = 0; i < n; ++i) depth[i] = -xy[2 * i + 1];
  out.perm.resize(n);
  for (int i = 0; i < n; ++i) out.perm[i] = i;
  std::stable_sort(out.perm.begin(), out.perm.end(),
                   [&](int a, int b) { return depth[a] < depth[b]; });
  std::vector<double> ds(n);
  for (int i = 0; i < n; ++i) ds[i] = depth[out.perm[i]];
  out.kcut.assign(2 * (size_t)q, n);
  out.jr.assign(4 * (size_t)n, 0);
  const double dmin = n > 0 ? ds[0] : 0.0;
  const double kmin = std::min(md.kp, md.ks);
  const bool on = eps > 0.0 && n > 0 && dmin > 0.0;
  const double thr = on ? bound_peak(2.0 * dmin, pmax, kmin) + std::log(eps) : 0.0;
  double kept = 0.0;
  for (int j = 0; j < q; ++j) {
    const cd x = nodes.xi[j];
    const double t = std::fabs(x.real());
    const bool real_node = x.imag() == 0.0;
    const double ap = t > md.kp ? std::sqrt((t - md.kp) * (t + md.kp)) : 0.0;
    const double as = t > md.ks ? std::sqrt((t - md.ks) * (t + md.ks)) : 0.0;
    const double amp = pmax * std::log(2.0 * t / kmin + 1.0);
    const double other = amp - std::min(ap, as) * std::min(dmin, std::max(dother, 0.0));
    for (int w = 0; w < 2; ++w) {
      const double a = w ? as : ap;
      int c = n;
      if (on && real_node && a > 0.0) {
        const double dcut = (amp + other - thr) / a;
        c = (int)(std::upper_bound(ds.begin(), ds.end(), dcut) - ds.begin());
      }
      out.kcut[(size_t)w * q + j] = c;
      kept += c;
    }
  }
  out.kept = (q > 0 && n > 0) ? kept / (2.0 * q * (double)n) : 1.0;
  // node hull of every particle: particle i is kept by node j iff i < kcut
  for (int w = 0; w < 2; ++w) {
    const int *kc = out.kcut.data() + (size_t)w * q;
    int *jr = out.jr.data();
    int hi = 0;
    for (int j = 0; j < q; ++j)
      for (; hi < kc[j]; ++hi) jr[2 * ((size_t)w * n + hi)] = j;
    hi = 0;
    for (int j = q - 1; j >= 0; --j)
      for (; hi < kc[j]; ++hi) jr[2 * ((size_t)w * n + hi) + 1] = j + 1;
  }
}

// ---------------------------------------------------------------------------
// Welded interface, one Fourier mode (Section 3.2, written for potentials).
// A potential e^{i xi x + q y} in (lambda, mu) gives (u1, u2, t1, t2) with
// t = T_y u: P: (i xi, q, 2 mu i xi q, (lambda + 2 mu) q^2 - lambda xi^2),
//            S: (-q, i xi, -mu (q^2 + xi^2), 2 mu i xi q).
static void pcol(cd xi, cd q, double lam, double mu, cd c[4]) {
  const cd I(0.0, 1.0);
  c[0] = I * xi;
  c[1] = q;
  c[2] = 2.0 * mu * I * xi * q;
  c[3] = (lam + 2.0 * mu) * q * q - lam * xi * xi;
}
static void scol(cd xi, cd q, double lam, double mu, cd c[4]) {
  const cd I(0.0, 1.0);
  c[0] = -q;
  c[1] = I * xi;
  c[2] = -mu * (q * q + xi * xi);
  c[3] = 2.0 * mu * I * xi * q;
}

void node_s(cd xi, double bp, double d, const Media &md, cd out[4]) {
  const double ks_[4] = {md.kp, md.ks, md.kpb, md.ksb};
  for (int i = 0; i < 4; ++i) {
    const double k = ks_[i];
    if (bp != 0.0 && std::fabs(std::fabs(bp) - k) <= 1e-14 * k) {
      const double v = d * (2.0 * bp + d);
      out[i] = v > 0 ? cd(std::sqrt(v), 0.0) : cd(0.0, -std::sqrt(-v));
    } else {
      out[i] = branch_s(xi, k);
    }
  }
}

// Derivatives of the potential columns with respect to the substrate's
// Lame parameters: explicit dependence plus the dependence through q.
static void dpcol(cd xi, cd q, cd dq, double lam, double mu, int which, cd c[4]) {
  const cd I(0.0, 1.0);
  // d/dq: (0, 1, 2 mu i xi, 2 (lam + 2 mu) q)
  c[0] = 0.0;
  c[1] = dq;
  c[2] = 2.0 * mu * I * xi * dq;
  c[3] = 2.0 * (lam + 2.0 * mu) * q * dq;
  if (which == 0) {  // lambda
    c[3] += q * q - xi * xi;
  } else {           // mu
    c[2] += 2.0 * I * xi * q;
    c[3] += 2.0 * q * q;
  }
}
static void dscol(cd xi, cd q, cd dq, double mu, int which, cd c[4]) {
  const cd I(0.0, 1.0);
  // d/dq: (-1, 0, -2 mu q, 2 mu i xi)
  c[0] = -dq;
  c[1] = 0.0;
  c[2] = -2.0 * mu * q * dq;
  c[3] = 2.0 * mu * I * xi * dq;
  if (which == 1) {  // mu
    c[2] += -(q * q + xi * xi);
    c[3] += 2.0 * I * xi * q;
  }
}

int reflection(cd xi, const Media &md, cd R[4]) {
  cd s[4];
  node_s(xi, 0.0, 0.0, md, s);
  return reflection_s(xi, s, md, R);
}

// The four continuity conditions (u_x, u_y, t_xy, t_yy at y = 0, Section
// 3.2) for potentials at one xi.  Unknowns: host downgoing P, S (e^{+s y})
// and substrate upgoing P, S (e^{-s_b y}); M = [P_h(+s_p), S_h(+s_s),
// -P_b(-s_pb), -S_b(-s_sb)], X = M^{-1} B for the two columns of B.
static int interface_solve(cd xi, const cd s4[4], const Media &md, const cd B[4][2],
                           cd X[4][2]) {
  const cd sp = s4[0], ss = s4[1], spb = s4[2], ssb = s4[3];
  cd M[4][6];
  cd c[4];
  pcol(xi, sp, md.lam_h, md.mu_h, c);
  for (int r = 0; r < 4; ++r) M[r][0] = c[r];
  scol(xi, ss, md.lam_h, md.mu_h, c);
  for (int r = 0; r < 4; ++r) M[r][1] = c[r];
  pcol(xi, -spb, md.lam_b, md.mu_b, c);
  for (int r = 0; r < 4; ++r) M[r][2] = -c[r];
  scol(xi, -ssb, md.lam_b, md.mu_b, c);
  for (int r = 0; r < 4; ++r) M[r][3] = -c[r];
  for (int r = 0; r < 4; ++r) {
    M[r][4] = B[r][0];
    M[r][5] = B[r][1];
  }
  // Gaussian elimination with partial pivoting on the 4x4 block, 2 RHS.
  for (int k = 0; k < 4; ++k) {
    int piv = k;
    for (int r = k + 1; r < 4; ++r)
      if (std::abs(M[r][k]) > std::abs(M[piv][k])) piv = r;
    if (std::abs(M[piv][k]) == 0.0) return EMS_ERR_NUMERIC;
    if (piv != k)
      for (int cc = 0; cc < 6; ++cc) std::swap(M[k][cc], M[piv][cc]);
    for (int r = k + 1; r < 4; ++r) {
      const cd f = M[r][k] / M[k][k];
      for (int cc = k; cc < 6; ++cc) M[r][cc] -= f * M[k][cc];
    }
  }
  for (int col = 0; col < 2; ++col)
    for (int k = 3; k >= 0; --k) {
      cd s = M[k][4 + col];
      for (int cc = k + 1; cc < 4; ++cc) s -= M[k][cc] * X[cc][col];
      X[k][col] = s / M[k][k];
    }
  for (int k = 0; k < 4; ++k)
    for (int col = 0; col < 2; ++col)
      if (!std::isfinite(X[k][col].real()) || !std::isfinite(X[k][col].imag()))
        return EMS_ERR_NUMERIC;
  return EMS_OK;
}

// Waves from the host: a unit upgoing P (column 0) or S (column 1) potential
// e^{i xi x - s y}; R = host downgoing, T = substrate upgoing potentials.
int reflect_transmit_s(cd xi, const cd s4[4], const Media &md, cd R[4], cd T[4]) {
  cd B[4][2], c[4], X[4][2];
  pcol(xi, -s4[0], md.lam_h, md.mu_h, c);
  for (int r = 0; r < 4; ++r) B[r][0] = -c[r];
  scol(xi, -s4[1], md.lam_h, md.mu_h, c);
  for (int r = 0; r < 4; ++r) B[r][1] = -c[r];
  const int rc = interface_solve(xi, s4, md, B, X);
  if (rc) return rc;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      R[2 * a + b] = X[a][b];
      if (T) T[2 * a + b] = X[2 + a][b];
    }
  return EMS_OK;
}

int reflection_s(cd xi, const cd s4[4], const Media &md, cd R[4]) {
  return reflect_transmit_s(xi, s4, md, R, nullptr);
}

// Waves from the substrate (Section 7.3's plane-wave setup): a unit
// downgoing P (column 0) or S (column 1) potential e^{i xi x + s_b y}; the
// continuity conditions move it to the right-hand side.  Td = host
// downgoing (transmitted), Rb = substrate upgoing (reflected) potentials.
int from_substrate_s(cd xi, const cd s4[4], const Media &md, cd Td[4], cd Rb[4]) {
  cd B[4][2], c[4], X[4][2];
  pcol(xi, s4[2], md.lam_b, md.mu_b, c);
  for (int r = 0; r < 4; ++r) B[r][0] = c[r];
  scol(xi, s4[3], md.lam_b, md.mu_b, c);
  for (int r = 0; r < 4; ++r) B[r][1] = c[r];
  const int rc = interface_solve(xi, s4, md, B, X);
  if (rc) return rc;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      Td[2 * a + b] = X[a][b];
      if (Rb) Rb[2 * a + b] = X[2 + a][b];
    }
  return EMS_OK;
}

int from_substrate(cd xi, const Media &md, cd Td[4], cd Rb[4]) {
  cd s[4];
  node_s(xi, 0.0, 0.0, md, s);
  return from_substrate_s(xi, s, md, Td, Rb);
}

// ---------------------------------------------------------------------------
// Closed-form disk scattering matrix (Section 4.1, boundary condition imposed
// mode by mode).  Z in {J, H}; f(r) = Z_n(kp r), g(r) = Z_n(ks r).
// Rigid: rows (u_r, u_theta): grad phi -> (f', (i n / a) f),
//        grad^perp psi -> (-(i n / a) g, g').
// Traction-free: rows (sigma_rr, sigma_rtheta):
//   P: (-lambda kp^2 f + 2 mu f'', 2 mu (i n / a)(f' - f / a))
//   S: (-2 mu (i n / a)(g' - g / a), mu (g'' - g' / a + n^2 g / a^2)).
static void bessel_jy(int n, double x, double &J, double &Y) {
  const int an = std::abs(n);
  J = ::jn(an, x);
  Y = ::yn(an, x);
  if (n < 0 && (an & 1)) {
    J = -J;
    Y = -Y;
  }
}

static void zfun(bool hankel, int n, double z, cd &f0, cd &f1, cd &f2) {
  double Jm, Ym, J0, Y0, Jp, Yp;
  bessel_jy(n - 1, z, Jm, Ym);
  bessel_jy(n, z, J0, Y0);
  bessel_jy(n + 1, z, Jp, Yp);
  if (hankel) {
    f0 = cd(J0, Y0);
    f1 = 0.5 * (cd(Jm, Ym) - cd(Jp, Yp));
  } else {
    f0 = cd(J0, 0.0);
    f1 = cd(0.5 * (Jm - Jp), 0.0);
  }
  f2 = -f1 / z - (1.0 - double(n) * n / (z * z)) * f0;
}

static void bc_matrix(bool hankel, int n, double a, const Media &md, int bc, cd M[4]) {
  const cd I(0.0, 1.0);
  cd fp0, fp1, fp2, fs0, fs1, fs2;
  zfun(hankel, n, md.kp * a, fp0, fp1, fp2);
  zfun(hankel, n, md.ks * a, fs0, fs1, fs2);
  const cd f = fp0, df = md.kp * fp1, d2f = md.kp * md.kp * fp2;
  const cd g = fs0, dg = md.ks * fs1, d2g = md.ks * md.ks * fs2;
  const double nn = n;
  if (bc == 0) {
    M[0] = df;
    M[1] = -(I * nn / a) * g;
    M[2] = (I * nn / a) * f;
    M[3] = dg;
  } else {
    const double lam = md.lam_h, mu = md.mu_h;
    M[0] = -lam * md.kp * md.kp * f + 2.0 * mu * d2f;
    M[1] = -2.0 * mu * (I * nn / a) * (dg - g / a);
    M[2] = 2.0 * mu * (I * nn / a) * (df - f / a);
    M[3] = mu * (d2g - dg / a + nn * nn * g / (a * a));
  }
}

int disk_smatrix(const Media &md, double a, int p, int bc, std::vector<cd> &S) {
  const int N = 2 * p + 1, K = 2 * N;
  S.assign((size_t)K * K, cd(0.0, 0.0));
  for (int n = -p; n <= p; ++n) {
    cd J[4], H[4];
    bc_matrix(false, n, a, md, bc, J);
    bc_matrix(true, n, a, md, bc, H);
    const cd det = H[0] * H[3] - H[1] * H[2];
    if (std::abs(det) == 0.0) return EMS_ERR_NUMERIC;
    // -H^{-1} J
    const cd Hi[4] = {H[3] / det, -H[1] / det, -H[2] / det, H[0] / det};
    cd B[4];
    B[0] = -(Hi[0] * J[0] + Hi[1] * J[2]);
    B[1] = -(Hi[0] * J[1] + Hi[1] * J[3]);
    B[2] = -(Hi[2] * J[0] + Hi[3] * J[2]);
    B[3] = -(Hi[2] * J[1] + Hi[3] * J[3]);
    const int k = n + p;
    S[(size_t)k * K + k] = B[0];
    S[(size_t)k * K + N + k] = B[1];
    S[(size_t)(N + k) * K + k] = B[2];
    S[(size_t)(N + k) * K + N + k] = B[3];
  }
  return EMS_OK;
}

// R(xi) and its derivatives with respect to the substrate's lambda and mu
// (Section 3.2 system differentiated): with M X = -B, only the substrate
// columns of M depend on (lambda_b, mu_b), explicitly and through
// s_pb = sqrt(xi^2 - kpb^2), s_sb = sqrt(xi^2 - ksb^2), kpb^2 = w^2 rho_b /
// (lambda_b + 2 mu_b), ksb^2 = w^2 rho_b / mu_b; then dX = -M^{-1} (dM) X.
// dR[0..3]: d/dlambda_b, dR[4..7]: d/dmu_b (row-major 2x2 blocks).
int reflection_deriv_s(cd xi, const cd s4[4], const Media &md, cd R[4], cd dR[8]) {
  const cd sp = s4[0], ss = s4[1], spb = s4[2], ssb = s4[3];
  cd M[4][4], B[4][2], c[4];
  auto put = [&](int col, const cd *v, double sg) {
    for (int r = 0; r < 4; ++r) M[r][col] = sg * v[r];
  };
  pcol(xi, sp, md.lam_h, md.mu_h, c);
  put(0, c, 1.0);
  scol(xi, ss, md.lam_h, md.mu_h, c);
  put(1, c, 1.0);
  pcol(xi, -spb, md.lam_b, md.mu_b, c);
  put(2, c, -1.0);
  scol(xi, -ssb, md.lam_b, md.mu_b, c);
  put(3, c, -1.0);
  pcol(xi, -sp, md.lam_h, md.mu_h, c);
  for (int r = 0; r < 4; ++r) B[r][0] = -c[r];
  scol(xi, -ss, md.lam_h, md.mu_h, c);
  for (int r = 0; r < 4; ++r) B[r][1] = -c[r];
  // LU with partial pivoting (row permutation kept in perm)
  int perm[4] = {0, 1, 2, 3};
  cd LU[4][4];
  for (int r = 0; r < 4; ++r)
    for (int cc = 0; cc < 4; ++cc) LU[r][cc] = M[r][cc];
  for (int k = 0; k < 4; ++k) {
    int piv = k;
    for (int r = k + 1; r < 4; ++r)
      if (std::abs(LU[r][k]) > std::abs(LU[piv][k])) piv = r;
    if (std::abs(LU[piv][k]) == 0.0) return EMS_ERR_NUMERIC;
    if (piv != k) {
      for (int cc = 0; cc < 4; ++cc) std::swap(LU[k][cc], LU[piv][cc]);
      std::swap(perm[k], perm[piv]);
    }
    for (int r = k + 1; r < 4; ++r) {
      LU[r][k] /= LU[k][k];
      for (int cc = k + 1; cc < 4; ++cc) LU[r][cc] -= LU[r][k] * LU[k][cc];
    }
  }
  auto solve = [&](const cd rhs[4], cd x[4]) {
    cd y[4];
    for (int r = 0; r < 4; ++r) {
      cd v = rhs[perm[r]];
      for (int cc = 0; cc < r; ++cc) v -= LU[r][cc] * y[cc];
      y[r] = v;
    }
    for (int r = 3; r >= 0; --r) {
      cd v = y[r];
      for (int cc = r + 1; cc < 4; ++cc) v -= LU[r][cc] * x[cc];
      x[r] = v / LU[r][r];
    }
  };
  cd X[2][4];
  for (int col = 0; col < 2; ++col) {
    const cd rhs[4] = {B[0][col], B[1][col], B[2][col], B[3][col]};
    solve(rhs, X[col]);
  }
  R[0] = X[0][0];
  R[1] = X[1][0];
  R[2] = X[0][1];
  R[3] = X[1][1];
  const double lp = md.lam_b + 2.0 * md.mu_b;
  const double kpb2 = md.kpb * md.kpb, ksb2 = md.ksb * md.ksb;
  for (int which = 0; which < 2; ++which) {
    // ds/dtheta (s = sqrt(xi^2 - k^2), k^2 depends on theta)
    const cd dspb = (which == 0 ? 1.0 : 2.0) * kpb2 / (2.0 * spb * lp);
    const cd dssb = which == 0 ? cd(0.0) : cd(ksb2 / (2.0 * ssb * md.mu_b));
    cd dM2[4], dM3[4];
    // columns 2, 3 are -pcol(xi, -spb), -scol(xi, -ssb): q = -s, dq = -ds
    dpcol(xi, -spb, -dspb, md.lam_b, md.mu_b, which, dM2);
    dscol(xi, -ssb, -dssb, md.mu_b, which, dM3);
    for (int col = 0; col < 2; ++col) {
      cd rhs[4], dx[4];
      for (int r = 0; r < 4; ++r) rhs[r] = dM2[r] * X[col][2] + dM3[r] * X[col][3];  // -(dM) X
      solve(rhs, dx);
      // row-major 2x2: dR[row][col]
      dR[4 * which + 0 * 2 + col] = dx[0];
      dR[4 * which + 1 * 2 + col] = dx[1];
    }
  }
  for (int i = 0; i < 8; ++i)
    if (!std::isfinite(dR[i].real()) || !std::isfinite(dR[i].imag())) return EMS_ERR_NUMERIC;
  return EMS_OK;
}

int reflection_deriv(cd xi, const Media &md, cd R[4], cd dR[8]) {
  cd s[4];
  node_s(xi, 0.0, 0.0, md, s);
  return reflection_deriv_s(xi, s, md, R, dR);
}

}  // namespace ems
