// Host set-up of the free-space fast multipole method (two scalar Helmholtz
// FMMs, kp acting on the alpha coefficients and ks on beta; the paper cites
// the FMM for the particle translations without describing it, Section 4.2).
//
// Uniform quadtree on the bounding square, leaf side chosen for about
// `leaf` particles per box.  Above the leaves, levels are kept up to a top
// level with at most `top_boxes` occupied boxes; on the top level every pair
// of non-adjacent boxes interacts directly (no coarser levels).  Below it the
// standard interaction list (children of the parent's neighbours that are not
// neighbours) is used.  Pairs of particles in adjacent leaves are summed
// directly (near field).
//
// Every translation is a Toeplitz product out_k = sum_j s_{j-k} in_j:
//   P2M, M2M, L2L, L2P: s_nu = J_nu(k rho) e^{i nu phi}, (rho, phi) the
//     polar form of (destination centre - source centre) for P2M / M2M and of
//     (destination - source) for L2L / L2P (Graf's theorem for J and H);
//   M2L: s_nu = t_{-nu} with t_nu = H_nu(k d) e^{-i nu (th - pi)}, the same
//     symbol as the particle-to-particle translation of Section 4.2.
// The symbols are tabulated here once per geometry and frequency.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>

#include "ems_internal.h"

namespace ems {

namespace {

// J_nu(x), nu = 0..L (Miller's backward recurrence normalised by
// J_0 + 2 sum J_2k = 1; forward recurrence when L < x is also stable but
// the backward sweep is used throughout for simplicity).
void besselj_seq(int L, double x, std::vector<double> &J) {
  J.assign(L + 1, 0.0);
  if (x < 1e-300) {
    J[0] = 1.0;
    return;
  }
  const int N = std::max(L, (int)std::ceil(x)) + 40 + (int)std::ceil(std::sqrt(60.0 * std::max((double)L, x)));
  std::vector<double> t(N + 2, 0.0);
  t[N + 1] = 0.0;
  t[N] = 1e-300;
  for (int n = N; n >= 1; --n) {
    t[n - 1] = (2.0 * n / x) * t[n] - t[n + 1];
    if (std::fabs(t[n - 1]) > 1e250) {
      for (int k = n - 1; k <= N; ++k) t[k] *= 1e-250;
    }
  }
  double s = t[0];
  for (int k = 2; k <= N; k += 2) s += 2.0 * t[k];
  for (int n = 0; n <= L; ++n) J[n] = t[n] / s;
}

// Y_nu(x), nu = 0..L by forward recurrence from Y_0, Y_1 (stable).
void bessely_seq(int L, double x, std::vector<double> &Y) {
  Y.assign(L + 1, 0.0);
  Y[0] = ::y0(x);
  if (L >= 1) Y[1] = ::y1(x);
  for (int n = 1; n < L; ++n) Y[n + 1] = (2.0 * n / x) * Y[n] - Y[n - 1];
}

// s_nu = J_nu(k rho) e^{i nu phi}, nu in [-L, L], appended to pool.
int64_t push_jsym(std::vector<cd> &pool, int L, double k, double rho, double phi) {
  std::vector<double> J;
  besselj_seq(L, k * rho, J);
  const int64_t base = (int64_t)pool.size();
  pool.resize(pool.size() + 2 * L + 1);
  for (int nu = 0; nu <= L; ++nu) {
    const cd e = std::polar(1.0, nu * phi);
    pool[base + L + nu] = J[nu] * e;
    // J_{-nu} e^{-i nu phi} = (-1)^nu J_nu conj(e)
    pool[base + L - nu] = ((nu & 1) ? -J[nu] : J[nu]) * std::conj(e);
  }
  return base;
}

// M2L symbol in the s_{j-k} convention: s_nu = t_{-nu},
// t_nu = H_nu(k d) e^{-i nu (th - pi)}, H_{-nu} = (-1)^nu H_nu.
int64_t push_hsym(std::vector<cd> &pool, int L, double k, double d, double th) {
  std::vector<double> J, Y;
  besselj_seq(L, k * d, J);
  bessely_seq(L, k * d, Y);
  const int64_t base = (int64_t)pool.size();
  pool.resize(pool.size() + 2 * L + 1);
  for (int nu = 0; nu <= L; ++nu) {
    const cd H(J[nu], Y[nu]);
    const cd e = std::polar(1.0, -nu * (th - 3.14159265358979323846));
    const cd t_pos = H * e;                                     // t_{+nu}
    const cd t_neg = ((nu & 1) ? -H : H) * std::conj(e);        // t_{-nu}
    pool[base + L - nu] = t_pos;  // s_{-nu} = t_{nu}
    pool[base + L + nu] = t_neg;  // s_{+nu} = t_{-nu}
  }
  return base;
}

}  // namespace

int fmm_order(double k, double side, int p, double digits) {
  const double r = side / std::sqrt(2.0), kr = k * r;
  const int hf = p + (int)std::ceil(kr + 1.8 * std::cbrt(std::max(kr, 1.0)) * std::pow(digits, 2.0 / 3.0)) + 2;
  const int lf = p + (int)std::ceil(digits * std::log(10.0) / std::log(1.0 / 0.55));
  return std::max(hf, lf);
}

int build_fmm(const ems_handle *h, FmmPlan &F, std::string &err) {
  F = FmmPlan();
  const int n = h->n;
  const std::vector<double> &xy = h->xy;
  double xlo = 1e300, xhi = -1e300, ylo = 1e300, yhi = -1e300;
  for (int i = 0; i < n; ++i) {
    xlo = std::min(xlo, xy[2 * i]);
    xhi = std::max(xhi, xy[2 * i]);
    ylo = std::min(ylo, xy[2 * i + 1]);
    yhi = std::max(yhi, xy[2 * i + 1]);
  }
  const double S0 = std::max(xhi - xlo, yhi - ylo) * 1.0001 + 1e-9;
  const double ox = 0.5 * (xlo + xhi) - 0.5 * S0, oy = 0.5 * (ylo + yhi) - 0.5 * S0;
  const double area = std::max((xhi - xlo) * (yhi - ylo), 1e-9);
  const double dens = n / area;
  const double side_leaf = std::sqrt(std::max(1.0, (double)h->fmm_leaf) / dens);
  int Lf = std::max(2, (int)std::lround(std::log2(S0 / side_leaf)));
  Lf = std::min(Lf, 14);
  auto box_of = [&](int i, int l, int &bx, int &by) {
    const double side = S0 / (double)(1 << l);
    bx = std::min((1 << l) - 1, std::max(0, (int)std::floor((xy[2 * i] - ox) / side)));
    by = std::min((1 << l) - 1, std::max(0, (int)std::floor((xy[2 * i + 1] - oy) / side)));
  };
  int Lt = Lf;
  while (Lt > 2) {
    std::map<std::pair<int, int>, int> occ;
    for (int i = 0; i < n; ++i) {
      int bx, by;
      box_of(i, Lt, bx, by);
      occ[{bx, by}] = 1;
    }
    if ((int)occ.size() <= h->fmm_top) break;
    --Lt;
  }
  F.Lf = Lf;
  F.Lt = Lt;
  F.S0 = S0;
  // occupied boxes per level
  const int nl = Lf - Lt + 1;
  F.levels.resize(nl);
  std::vector<std::map<std::pair<int, int>, int>> index(nl);
  std::vector<int> leaf_of(n);
  for (int li = nl - 1; li >= 0; --li) {
    const int l = Lt + li;
    for (int i = 0; i < n; ++i) {
      int bx, by;
      box_of(i, l, bx, by);
      auto key = std::make_pair(bx, by);
      auto it = index[li].find(key);
      int id;
      if (it == index[li].end()) {
        id = (int)F.levels[li].bx.size();
        index[li][key] = id;
        F.levels[li].bx.push_back(bx);
        F.levels[li].by.push_back(by);
      } else {
        id = it->second;
      }
      if (l == Lf) leaf_of[i] = id;
    }
    const double side = S0 / (double)(1 << l);
    for (int w = 0; w < 2; ++w) {
      const double k = w == 0 ? h->md.kp : h->md.ks;
      F.levels[li].P[w] = fmm_order(k, side, h->pmax, h->fmm_digits);
    }
    F.levels[li].side = side;
  }
  auto center = [&](int li, int id, double &cx, double &cy) {
    const double side = F.levels[li].side;
    cx = ox + (F.levels[li].bx[id] + 0.5) * side;
    cy = oy + (F.levels[li].by[id] + 0.5) * side;
  };
  // expansion storage offsets (complex elements, per right-hand side)
  int64_t eo = 0;
  for (int w = 0; w < 2; ++w)
    for (int li = 0; li < nl; ++li) {
      F.levels[li].off[w] = eo;
      eo += (int64_t)F.levels[li].bx.size() * (2 * F.levels[li].P[w] + 1);
    }
  F.exp_len = eo;
  std::vector<cd> pool;
  // ---- near lists: partners in adjacent leaves ----------------------------
  {
    const int nleaf = (int)F.levels[nl - 1].bx.size();
    std::vector<std::vector<int>> members(nleaf);
    for (int i = 0; i < n; ++i) members[leaf_of[i]].push_back(i);
    F.nbr_ptr.assign(n + 1, 0);
    F.nbr_idx.clear();
    for (int i = 0; i < n; ++i) {
      const int b = leaf_of[i];
      const int bx = F.levels[nl - 1].bx[b], by = F.levels[nl - 1].by[b];
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy) {
          auto it = index[nl - 1].find({bx + dx, by + dy});
          if (it == index[nl - 1].end()) continue;
          for (int j : members[it->second])
            if (j != i) F.nbr_idx.push_back(j);
        }
      F.nbr_ptr[i + 1] = (int)F.nbr_idx.size();
    }
  }
  // ---- task lists ------------------------------------------------------------
  auto new_launch = [&](int in_kind, int out_kind, int accumulate) {
    F.launches.emplace_back();
    FmmLaunch &L = F.launches.back();
    L.in_kind = in_kind;
    L.out_kind = out_kind;
    L.accumulate = accumulate;
    L.ptr.push_back(0);
    return (int)F.launches.size() - 1;
  };
  auto add_task = [&](FmmLaunch &L, int64_t in_base, int in_P, int64_t sym, int symL, int sgn) {
    L.in_base.push_back(in_base);
    L.in_P.push_back(in_P);
    L.sym_base.push_back(sym);
    L.sym_L.push_back(symL);
    L.sgn.push_back(sgn);
  };
  auto end_output = [&](FmmLaunch &L, int64_t out_base, int out_P) {
    L.out_base.push_back(out_base);
    L.out_P.push_back(out_P);
    L.ptr.push_back((int)L.in_base.size());
  };
  const int leaf_li = nl - 1;
  // P2M: leaf multipoles from the particles (in = x, out = multipoles)
  {
    const int id = new_launch(0, 1, 0);
    FmmLaunch &L = F.launches[id];
    const int nleaf = (int)F.levels[leaf_li].bx.size();
    std::vector<std::vector<int>> members(nleaf);
    for (int i = 0; i < n; ++i) members[leaf_of[i]].push_back(i);
    F.part_sym.assign(2 * (size_t)n, 0);
    for (int w = 0; w < 2; ++w) {
      const double k = w == 0 ? h->md.kp : h->md.ks;
      const int P = F.levels[leaf_li].P[w];
      for (int b = 0; b < nleaf; ++b) {
        double cx, cy;
        center(leaf_li, b, cx, cy);
        for (int i : members[b]) {
          const int symL = P + h->pmax;
          const double dx = cx - xy[2 * i], dy = cy - xy[2 * i + 1];
          const int64_t s = push_jsym(pool, symL, k, std::hypot(dx, dy), std::atan2(dy, dx));
          F.part_sym[2 * (size_t)i + w] = s;
          add_task(L, h->off[i] + w * (2 * h->p[i] + 1), h->p[i], s, symL, 1);
        }
        end_output(L, F.levels[leaf_li].off[w] + (int64_t)b * (2 * P + 1), P);
      }
    }
  }
  // M2M: level li -> li - 1
  for (int li = nl - 1; li >= 1; --li) {
    const int id = new_launch(1, 1, 0);
    FmmLaunch &L = F.launches[id];
    const int npar = (int)F.levels[li - 1].bx.size();
    std::vector<std::vector<int>> kids(npar);
    for (int b = 0; b < (int)F.levels[li].bx.size(); ++b) {
      auto it = index[li - 1].find({F.levels[li].bx[b] >> 1, F.levels[li].by[b] >> 1});
      kids[it->second].push_back(b);
    }
    for (int w = 0; w < 2; ++w) {
      const double k = w == 0 ? h->md.kp : h->md.ks;
      const int Pc = F.levels[li].P[w], Pp = F.levels[li - 1].P[w];
      std::map<int, int64_t> sym_of;  // child position -> symbol
      for (int pb = 0; pb < npar; ++pb) {
        double px, py;
        center(li - 1, pb, px, py);
        for (int c : kids[pb]) {
          double cx, cy;
          center(li, c, cx, cy);
          const int pos = (F.levels[li].bx[c] & 1) + 2 * (F.levels[li].by[c] & 1);
          auto it = sym_of.find(pos);
          int64_t s;
          if (it == sym_of.end()) {
            s = push_jsym(pool, Pc + Pp, k, std::hypot(px - cx, py - cy), std::atan2(py - cy, px - cx));
            sym_of[pos] = s;
          } else {
            s = it->second;
          }
          add_task(L, F.levels[li].off[w] + (int64_t)c * (2 * Pc + 1), Pc, s, Pc + Pp, 1);
        }
        end_output(L, F.levels[li - 1].off[w] + (int64_t)pb * (2 * Pp + 1), Pp);
      }
    }
  }
  // M2L per level, top down, as matrix products on the matrix cores (one
  // launch marker per level covering both waves), then L2L from the parent
  // local as a task launch that accumulates onto it (in = loc, out = loc).
  for (int li = 0; li < nl; ++li) {
    const int nb = (int)F.levels[li].bx.size();
    // source boxes of every target: all non-adjacent boxes on the top level,
    // the interaction list (children of the parent's neighbours that are not
    // neighbours) below it
    std::vector<std::vector<int>> srcs(nb);
    for (int b = 0; b < nb; ++b) {
      const int bx = F.levels[li].bx[b], by = F.levels[li].by[b];
      if (li == 0) {
        for (int s = 0; s < nb; ++s)
          if (std::max(std::abs(F.levels[li].bx[s] - bx), std::abs(F.levels[li].by[s] - by)) > 1)
            srcs[b].push_back(s);
      } else {
        const int pbx = bx >> 1, pby = by >> 1;
        for (int dx = -1; dx <= 1; ++dx)
          for (int dy = -1; dy <= 1; ++dy)
            for (int ex = 0; ex < 2; ++ex)
              for (int ey = 0; ey < 2; ++ey) {
                const int sx = 2 * (pbx + dx) + ex, sy = 2 * (pby + dy) + ey;
                if (std::max(std::abs(sx - bx), std::abs(sy - by)) <= 1) continue;
                auto it = index[li].find({sx, sy});
                if (it != index[li].end()) srcs[b].push_back(it->second);
              }
      }
      F.n_m2l += 2 * (int64_t)srcs[b].size();
    }
    // column tiles: boxes grouped by position in the parent (one group on
    // the top level), row-major order inside a group
    std::vector<int> order(nb);
    for (int b = 0; b < nb; ++b) order[b] = b;
    auto cls = [&](int b) {
      return li == 0 ? 0 : (F.levels[li].bx[b] & 1) + 2 * (F.levels[li].by[b] & 1);
    };
    std::sort(order.begin(), order.end(), [&](int a, int b) {
      const int ca = cls(a), cb = cls(b);
      if (ca != cb) return ca < cb;
      if (F.levels[li].by[a] != F.levels[li].by[b]) return F.levels[li].by[a] < F.levels[li].by[b];
      return F.levels[li].bx[a] < F.levels[li].bx[b];
    });
    std::vector<std::vector<int>> tiles;
    for (int k = 0; k < nb;) {
      std::vector<int> t;
      const int c0 = cls(order[k]);
      while (k < nb && (int)t.size() < kM2lCols && cls(order[k]) == c0) t.push_back(order[k++]);
      tiles.push_back(t);
    }
    if (li == 0) {
      // top level: every non-adjacent pair, nearly every pair its own offset,
      // so column tiles would be sparse; the Toeplitz task kernel runs it
      const int id = new_launch(1, 2, 0);
      FmmLaunch &L = F.launches[id];
      for (int w = 0; w < 2; ++w) {
        const double k = w == 0 ? h->md.kp : h->md.ks;
        const int P = F.levels[li].P[w];
        std::map<std::pair<int, int>, int64_t> sym_of;
        for (int b = 0; b < nb; ++b) {
          double cx, cy;
          center(li, b, cx, cy);
          for (int s : srcs[b]) {
            const std::pair<int, int> key(F.levels[li].bx[s] - F.levels[li].bx[b],
                                          F.levels[li].by[s] - F.levels[li].by[b]);
            auto it = sym_of.find(key);
            int64_t sy;
            if (it == sym_of.end()) {
              double sx_, sy_;
              center(li, s, sx_, sy_);
              sy = push_hsym(pool, 2 * P, k, std::hypot(cx - sx_, cy - sy_), std::atan2(cy - sy_, cx - sx_));
              sym_of[key] = sy;
            } else {
              sy = it->second;
            }
            add_task(L, F.levels[li].off[w] + (int64_t)s * (2 * P + 1), P, sy, 2 * P, 1);
          }
          end_output(L, F.levels[li].off[w] + (int64_t)b * (2 * P + 1), P);
        }
      }
      continue;
    }
    F.launches.emplace_back();
    F.launches.back().gemm_level = li;
    F.launches.back().ptr.push_back(0);
    M2lPlan &Q = F.m2l;
    for (int w = 0; w < 2; ++w) {
      const double k = w == 0 ? h->md.kp : h->md.ks;
      const int P = F.levels[li].P[w], N = 2 * P + 1;
      const int g = (int)Q.g_P.size();
      Q.g_li.push_back(li);
      Q.g_w.push_back(w);
      Q.g_P.push_back(P);
      Q.g_nb.push_back(nb);
      Q.g_off.push_back(F.levels[li].off[w]);
      Q.g_item0.push_back((int)Q.it_g.size());
      double flops = 0.0, symmax = 0.0;
      std::map<std::pair<int, int>, int64_t> sym_of;
      auto sym_at = [&](int b, int s) {
        const std::pair<int, int> key(F.levels[li].bx[s] - F.levels[li].bx[b],
                                      F.levels[li].by[s] - F.levels[li].by[b]);
        auto it = sym_of.find(key);
        if (it != sym_of.end()) return it->second;
        double cx, cy, sx_, sy_;
        center(li, b, cx, cy);
        center(li, s, sx_, sy_);
        const int64_t base = push_hsym(pool, 2 * P, k, std::hypot(cx - sx_, cy - sy_),
                                       std::atan2(cy - sy_, cx - sx_));
        for (int nu = 0; nu <= 4 * P; ++nu) symmax = std::max(symmax, std::abs(pool[base + nu]));
        sym_of[key] = base + 2 * P;  // index of s_0
        return base + 2 * P;
      };
      // tiles of this product with their entries
      std::vector<int> t0s, t1s;  // entry range per tile
      const int tile_base = (int)Q.tile_ptr.size() == 0 ? 0 : (int)Q.tile_ptr.size() - 1;
      if (Q.tile_ptr.empty()) Q.tile_ptr.push_back(0);
      int max_ent = 1;
      for (const auto &t : tiles) {
        std::map<std::pair<int, int>, std::vector<int>> ents;
        for (int c = 0; c < (int)t.size(); ++c) {
          const int b = t[c];
          for (int s : srcs[b]) {
            const std::pair<int, int> key(F.levels[li].bx[s] - F.levels[li].bx[b],
                                          F.levels[li].by[s] - F.levels[li].by[b]);
            auto &v = ents[key];
            if (v.empty()) v.assign(kM2lCols, -1);
            v[c] = s;
            flops += 8.0 * N * N;
          }
        }
        for (auto &kv : ents) {
          int first = -1;
          for (int c = 0; c < kM2lCols && first < 0; ++c)
            if (kv.second[c] >= 0) first = c;
          Q.ent_sym.push_back(sym_at(t[first], kv.second[first]));
          Q.ent_src.insert(Q.ent_src.end(), kv.second.begin(), kv.second.end());
        }
        Q.tile_ptr.push_back((int)Q.ent_sym.size());
        for (int c = 0; c < kM2lCols; ++c) Q.tile_box.push_back(c < (int)t.size() ? t[c] : -1);
        max_ent = std::max(max_ent, (int)ents.size());
      }
      // entry groups: about two wavefronts per SIMD (1024 SIMDs); more groups
      // would cost partial slots (G nb N complex per product and RHS)
      const int nrt = (N + 15) / 16, nt = (int)tiles.size();
      const int nit = (nrt + kM2lRowTiles - 1) / kM2lRowTiles;  // items per (tile, group)
      const int G = std::max(1, std::min(max_ent, (2048 + nit * nt - 1) / std::max(1, nit * nt)));
      Q.g_G.push_back(G);
      Q.g_poff.push_back(G > 1 ? Q.part_len : 0);
      if (G > 1) Q.part_len += (int64_t)G * nb * N;
      for (int ti = 0; ti < nt; ++ti) {
        const int tid = tile_base + ti;
        const int e0 = Q.tile_ptr[tid], ne = Q.tile_ptr[tid + 1] - e0;
        for (int gr = 0; gr < G; ++gr) {
          const int a0 = e0 + (int)((int64_t)ne * gr / G), a1 = e0 + (int)((int64_t)ne * (gr + 1) / G);
          for (int rt = 0; rt < nrt; rt += kM2lRowTiles) {
            Q.it_g.push_back(g);
            Q.it_rt.push_back(rt);
            Q.it_tile.push_back(tid);
            Q.it_e0.push_back(a0);
            Q.it_e1.push_back(a1);
            Q.it_slot.push_back(G > 1 ? gr : -1);
          }
        }
      }
      Q.g_flops.push_back(flops);
      Q.g_symmax.push_back(symmax);
      F.launches.back().flops += flops;
    }
    if (li > 0) {
      const int id = new_launch(1, 2, 1);
      FmmLaunch &L = F.launches[id];
      for (int w = 0; w < 2; ++w) {
        const double k = w == 0 ? h->md.kp : h->md.ks;
        const int P = F.levels[li].P[w];
        const int Pp = F.levels[li - 1].P[w];
        std::map<int, int64_t> l2l_of;
        for (int b = 0; b < nb; ++b) {
          const int bx = F.levels[li].bx[b], by = F.levels[li].by[b];
          double cx, cy;
          center(li, b, cx, cy);
          // L2L from the parent local (in = loc): marked by sgn = 2
          auto it = index[li - 1].find({bx >> 1, by >> 1});
          const int pb = it->second;
          const int pos = (bx & 1) + 2 * (by & 1);
          auto jt = l2l_of.find(pos);
          int64_t s;
          if (jt == l2l_of.end()) {
            double px, py;
            center(li - 1, pb, px, py);
            s = push_jsym(pool, Pp + P, k, std::hypot(cx - px, cy - py), std::atan2(cy - py, cx - px));
            l2l_of[pos] = s;
          } else {
            s = jt->second;
          }
          add_task(L, F.levels[li - 1].off[w] + (int64_t)pb * (2 * Pp + 1), Pp, s, Pp + P, 2);
          end_output(L, F.levels[li].off[w] + (int64_t)b * (2 * P + 1), P);
        }
      }
    }
  }
  // L2P: particle locals from the leaf locals (in = loc, out = free part,
  // accumulate onto the near field).  Symbol of (x_m - c) = J e^{i nu (phi + pi)}
  // = (-1)^nu times the P2M symbol: sgn = -1.
  {
    const int id = new_launch(2, 3, 1);
    FmmLaunch &L = F.launches[id];
    for (int w = 0; w < 2; ++w) {
      const int P = F.levels[leaf_li].P[w];
      for (int i = 0; i < n; ++i) {
        const int b = leaf_of[i];
        add_task(L, F.levels[leaf_li].off[w] + (int64_t)b * (2 * P + 1), P, F.part_sym[2 * (size_t)i + w],
                 P + h->pmax, -1);
        end_output(L, h->off[i] + w * (2 * h->p[i] + 1), h->p[i]);
      }
    }
  }
  for (auto &L : F.launches) {
    L.nout = (int)L.out_base.size();
    // (output, 192-row chunk) items: the task kernel's wavefront owns 64 x 3 rows
    int nchunk = 0, max_tasks = 1;
    for (int o = 0; o < L.nout; ++o) {
      nchunk += (2 * L.out_P[o] + 1 + kFmmRows - 1) / kFmmRows;
      max_tasks = std::max(max_tasks, L.ptr[o + 1] - L.ptr[o]);
    }
    // split task lists when there are too few items to fill the chip
    constexpr int kTargetItems = 4096;
    const int G = std::max(1, std::min({16, max_tasks, (kTargetItems + nchunk - 1) / std::max(1, nchunk)}));
    L.nslot = 0;
    for (int o = 0; o < L.nout; ++o) {
      const int rows = 2 * L.out_P[o] + 1;
      const int t0 = L.ptr[o], nt = L.ptr[o + 1] - L.ptr[o];
      const int g = std::max(1, std::min(G, nt));
      for (int c = 0; c * kFmmRows < rows; ++c) {
        if (g > 1) {
          L.red_out.push_back(o);
          L.red_row0.push_back(c * kFmmRows);
          L.red_slot0.push_back(L.nslot);
          L.red_g.push_back(g);
        }
        for (int k = 0; k < g; ++k) {
          L.item_out.push_back(o);
          L.item_row0.push_back(c * kFmmRows);
          L.item_t0.push_back(t0 + (int)((int64_t)nt * k / g));
          L.item_t1.push_back(t0 + (int)((int64_t)nt * (k + 1) / g));
          L.item_slot.push_back(g > 1 ? L.nslot++ : -1);
        }
      }
    }
    F.max_slots = std::max(F.max_slots, L.nslot);
    for (int t = 0; t < (int)L.in_P.size(); ++t) L.max_in_P = std::max(L.max_in_P, L.in_P[t]);
    for (int o = 0; o < L.nout; ++o) L.max_out_P = std::max(L.max_out_P, L.out_P[o]);
    if (L.gemm_level >= 0) continue;  // flops from the M2L plan
    L.flops = 0.0;
    for (int o = 0; o < L.nout; ++o)
      for (int t = L.ptr[o]; t < L.ptr[o + 1]; ++t)
        L.flops += 8.0 * (2 * L.out_P[o] + 1) * (2 * L.in_P[t] + 1);
  }
  F.pool = std::move(pool);
  // Bounds of every task against the buffers the kernel will touch.
  const int64_t npool = (int64_t)F.pool.size();
  for (const auto &L : F.launches) {
    const int64_t in_len = L.in_kind == 0 ? h->ncoef : F.exp_len;
    const int64_t out_len = L.out_kind == 3 ? h->ncoef : F.exp_len;
    for (int o = 0; o < L.nout; ++o) {
      if (L.out_base[o] < 0 || L.out_base[o] + 2 * L.out_P[o] >= out_len) {
        err = "fmm plan: output out of range";
        return EMS_ERR_NUMERIC;
      }
      for (int t = L.ptr[o]; t < L.ptr[o + 1]; ++t) {
        const int64_t il = L.sgn[t] == 2 ? F.exp_len : in_len;
        if (L.in_base[t] < 0 || L.in_base[t] + 2 * L.in_P[t] >= il || L.in_P[t] > L.max_in_P) {
          err = "fmm plan: input out of range";
          return EMS_ERR_NUMERIC;
        }
        if (L.sym_base[t] < 0 || L.sym_base[t] + 2 * L.sym_L[t] >= npool ||
            L.sym_L[t] < L.in_P[t] + L.out_P[o]) {
          err = "fmm plan: symbol out of range";
          return EMS_ERR_NUMERIC;
        }
      }
    }
    for (size_t it = 0; it < L.item_out.size(); ++it) {
      const int o = L.item_out[it];
      if (L.item_row0[it] >= 2 * L.out_P[o] + 1 || L.item_t0[it] < L.ptr[o] ||
          L.item_t1[it] > L.ptr[o + 1] || L.item_t0[it] > L.item_t1[it] ||
          L.item_slot[it] >= L.nslot) {
        err = "fmm plan: item out of range";
        return EMS_ERR_NUMERIC;
      }
    }
    for (size_t k = 0; k < L.red_out.size(); ++k)
      if (L.red_slot0[k] < 0 || L.red_slot0[k] + L.red_g[k] > L.nslot ||
          L.red_row0[k] >= 2 * L.out_P[L.red_out[k]] + 1) {
        err = "fmm plan: partial sum out of range";
        return EMS_ERR_NUMERIC;
      }
  }
  for (int v : F.nbr_idx)
    if (v < 0 || v >= n) {
      err = "fmm plan: near list out of range";
      return EMS_ERR_NUMERIC;
    }
  // the matrix-core M2L: boxes, sources, symbols and items inside their arrays
  {
    M2lPlan &Q = F.m2l;
    const int ng = (int)Q.g_P.size();
    Q.g_item0.push_back((int)Q.it_g.size());
    const int ntile = Q.tile_ptr.empty() ? 0 : (int)Q.tile_ptr.size() - 1;
    const int nent = (int)Q.ent_sym.size();
    if ((int64_t)Q.tile_box.size() != (int64_t)ntile * kM2lCols ||
        (int64_t)Q.ent_src.size() != (int64_t)nent * kM2lCols) {
      err = "fmm plan: M2L tile layout";
      return EMS_ERR_NUMERIC;
    }
    for (int g = 0; g < ng; ++g) {
      const int P = Q.g_P[g], N = 2 * P + 1, nbl = Q.g_nb[g];
      if (Q.g_off[g] < 0 || Q.g_off[g] + (int64_t)nbl * N > F.exp_len ||
          (Q.g_G[g] > 1 && Q.g_poff[g] + (int64_t)Q.g_G[g] * nbl * N > Q.part_len)) {
        err = "fmm plan: M2L product layout";
        return EMS_ERR_NUMERIC;
      }
      for (int it = Q.g_item0[g]; it < Q.g_item0[g + 1]; ++it) {
        const int tl = Q.it_tile[it];
        if (Q.it_g[it] != g || tl < 0 || tl >= ntile || Q.it_rt[it] < 0 ||
            16 * Q.it_rt[it] >= N || Q.it_e0[it] < Q.tile_ptr[tl] ||
            Q.it_e1[it] > Q.tile_ptr[tl + 1] || Q.it_e0[it] > Q.it_e1[it] ||
            Q.it_slot[it] >= Q.g_G[g] || (Q.g_G[g] > 1 && Q.it_slot[it] < 0)) {
          err = "fmm plan: M2L item out of range";
          return EMS_ERR_NUMERIC;
        }
        for (int c = 0; c < kM2lCols; ++c) {
          const int v = Q.tile_box[(int64_t)tl * kM2lCols + c];
          if (v < -1 || v >= nbl) {
            err = "fmm plan: M2L target out of range";
            return EMS_ERR_NUMERIC;
          }
        }
        for (int e = Q.it_e0[it]; e < Q.it_e1[it]; ++e) {
          if (Q.ent_sym[e] - 2 * P < 0 || Q.ent_sym[e] + 2 * P >= npool) {
            err = "fmm plan: M2L symbol out of range";
            return EMS_ERR_NUMERIC;
          }
          for (int c = 0; c < kM2lCols; ++c) {
            const int v = Q.ent_src[(int64_t)e * kM2lCols + c];
            if (v < -1 || v >= nbl) {
              err = "fmm plan: M2L source out of range";
              return EMS_ERR_NUMERIC;
            }
          }
        }
      }
    }
  }
  return EMS_OK;
}

}  // namespace ems
