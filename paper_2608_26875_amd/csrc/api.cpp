// C ABI of the library: handle life cycle, validation, set-up, the operator
// apply pipeline and the GMRES driver (Saad-Schultz GMRES named in Sections
// 4.2 and 5.2, restarted, CGS2 Arnoldi on the device, Givens on the host).
#include <algorithm>
#include <chrono>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <type_traits>

#include "ems_internal.h"

namespace ems {
hipError_t launch_s_apply(const ems_handle *h, const double2 *c, double2 *y, int nrhs,
                          bool adjoint, hipStream_t st);
hipError_t launch_incident_pw(const ems_handle *h, const double2 *pw, int nrhs, double2 *c,
                              hipStream_t st);
hipError_t launch_background(int nrhs, int npts, const double *pts, const double2 *comp,
                             double2 *u, hipStream_t st);
// V: workspace of 2 q (2 pmax + 1) complex values (the node powers).
hipError_t launch_point_local(const ems_handle *h, int q, const double2 *nd, const double2 *amp,
                              int nrhs, double2 *c, double2 *V, hipStream_t st);
hipError_t launch_point_field(const ems_handle *h, int q, const double2 *nd, const double2 *amp,
                              const double *src, int nrhs, int npts, const double *pts,
                              double2 *u, hipStream_t st);
}  // namespace ems

using ems::cd;

namespace {

int fail(ems_handle *h, int code, const std::string &msg) {
  if (h) h->err = msg;
  return code;
}

// The plane waves that make up the background field of one incident plane
// wave (Section 7.3, (bplan)): potentials A e^{i xi0 x + q y} in the host
// (layer 0) or the substrate (layer 1), P (kind 0) or S (kind 1); `up` marks
// a wave travelling towards y > 0 (q = -s), else q = +s.
struct PwComp {
  int layer, kind;
  bool up;
  cd A, q;
};
struct PwParts {
  double xi0 = 0.0;
  cd s4[4];
  std::vector<PwComp> comp;
};

int plane_wave_parts(const ems::Media &md, const ems_plane_wave &w, PwParts &out,
                     std::string &err) {
  const int wv = w.wave;
  if (wv < 0 || wv > 3) {
    err = "wave must be 0 (P) or 1 (SV) from the host, 2 (P) or 3 (SV) from the substrate";
    return EMS_ERR_ARG;
  }
  if (!(std::cos(w.angle) > 0)) {
    err = "plane wave must travel towards the interface (|angle| < pi/2)";
    return EMS_ERR_ARG;
  }
  const double k = wv == 0 ? md.kp : wv == 1 ? md.ks : wv == 2 ? md.kpb : md.ksb;
  const cd I(0.0, 1.0);
  const double xi0 = k * std::sin(w.angle);
  const cd A = 1.0 / (I * k);  // unit displacement
  out.xi0 = xi0;
  ems::node_s(cd(xi0, 0.0), 0.0, 0.0, md, out.s4);
  const cd *s = out.s4;
  out.comp.clear();
  cd X[4], Y[4];
  if (wv < 2) {
    if (ems::reflect_transmit_s(cd(xi0, 0.0), s, md, X, Y)) {
      err = "singular interface system at the incident wavenumber";
      return EMS_ERR_NUMERIC;
    }
    const int c = wv;  // incident column
    out.comp.push_back({0, c, true, A, -s[c]});
    out.comp.push_back({0, 0, false, X[0 + c] * A, s[0]});
    out.comp.push_back({0, 1, false, X[2 + c] * A, s[1]});
    out.comp.push_back({1, 0, true, Y[0 + c] * A, -s[2]});
    out.comp.push_back({1, 1, true, Y[2 + c] * A, -s[3]});
  } else {
    if (ems::from_substrate_s(cd(xi0, 0.0), s, md, X, Y)) {
      err = "singular interface system at the incident wavenumber";
      return EMS_ERR_NUMERIC;
    }
    const int c = wv - 2;
    out.comp.push_back({1, c, false, A, s[2 + c]});
    out.comp.push_back({1, 0, true, Y[0 + c] * A, -s[2]});
    out.comp.push_back({1, 1, true, Y[2 + c] * A, -s[3]});
    out.comp.push_back({0, 0, false, X[0 + c] * A, s[0]});
    out.comp.push_back({0, 1, false, X[2 + c] * A, s[1]});
  }
  return EMS_OK;
}

// Point sources in the substrate (Section 3.2): a node rule of their own and
// the per-node potentials.  The rule is the handle's Sommerfeld rule laid out
// for the source-to-target pairs: horizontal spread from the sources and the
// targets (particles or receivers), depth sums y0 + |y| (two stand-in points
// at half those sums, since the rule is designed for pairs of equal depth).
// Per node and source, with c = 1/(4 pi rho_b omega^2) and the substrate's s:
//   downgoing P potential  -c (i xi a1 + s_pb a2) e^{-s_pb y0} / s_pb e^{-i xi x0},
//   downgoing S potential   c (s_sb a1 - i xi a2) e^{-s_sb y0} / s_sb e^{-i xi x0}
// (the Green's tensor split into grad phi + grad^perp psi below the source);
// the host sees w Td of them, the substrate w Rb of them going up.
struct PointNodes {
  ems::NodeTable nt;
  std::vector<double2> nd;   // [q][5]: xi, s_p, s_s, s_pb, s_sb
  std::vector<double2> amp;  // [nsrc][q][4]: host P, S, substrate P, S
};

int point_nodes(ems_handle *h, const ems_point_source *src, int nsrc, double xlo, double xhi,
                double dlo, double dhi, PointNodes &out) {
  double slo = HUGE_VAL, shi = -HUGE_VAL;
  for (int r = 0; r < nsrc; ++r) {
    const ems_point_source &s = src[r];
    if (!std::isfinite(s.x0) || !std::isfinite(s.y0) || !std::isfinite(s.alpha1) ||
        !std::isfinite(s.alpha2))
      return fail(h, EMS_ERR_ARG, "non-finite point source");
    if (!(s.y0 > 0)) return fail(h, EMS_ERR_GEOMETRY, "point source not in the substrate (y0 > 0)");
    xlo = std::min(xlo, s.x0);
    xhi = std::max(xhi, s.x0);
    slo = std::min(slo, s.y0);
    shi = std::max(shi, s.y0);
  }
  const std::vector<double> xy = {xlo, -0.5 * (slo + dlo), xhi, -0.5 * (shi + dhi)};
  const std::vector<int> pp = {h->pmax, h->pmax};
  int rc = ems::build_nodes(h->somm, h->md, xy, pp, out.nt, h->err);
  if (rc) return rc;
  const int q = (int)out.nt.xi.size();
  out.nd.resize(5 * (size_t)q);
  out.amp.resize(4 * (size_t)q * nsrc);
  const ems::Media &md = h->md;
  const cd I(0.0, 1.0);
  const double c = 1.0 / (4.0 * 3.14159265358979323846 * md.rho_b * md.omega * md.omega);
  for (int j = 0; j < q; ++j) {
    const cd xi = out.nt.xi[j], w = out.nt.w[j];
    cd s4[4], Td[4], Rb[4];
    ems::node_s(xi, out.nt.bp[j], out.nt.d[j], md, s4);
    if (ems::from_substrate_s(xi, s4, md, Td, Rb))
      return fail(h, EMS_ERR_NUMERIC, "singular interface system at a point-source node");
    const cd v[5] = {xi, s4[0], s4[1], s4[2], s4[3]};
    for (int k = 0; k < 5; ++k) out.nd[5 * (size_t)j + k] = make_double2(v[k].real(), v[k].imag());
    for (int r = 0; r < nsrc; ++r) {
      const ems_point_source &s = src[r];
      const cd ph = std::exp(-I * xi * s.x0);
      const cd P = -c * (I * xi * s.alpha1 + s4[2] * s.alpha2) * std::exp(-s4[2] * s.y0) / s4[2] * ph;
      const cd S = c * (s4[3] * s.alpha1 - I * xi * s.alpha2) * std::exp(-s4[3] * s.y0) / s4[3] * ph;
      const cd a[4] = {w * (Td[0] * P + Td[1] * S), w * (Td[2] * P + Td[3] * S),
                       w * (Rb[0] * P + Rb[1] * S), w * (Rb[2] * P + Rb[3] * S)};
      for (int k = 0; k < 4; ++k) {
        if (!std::isfinite(a[k].real()) || !std::isfinite(a[k].imag()))
          return fail(h, EMS_ERR_NUMERIC, "non-finite point-source amplitude at a node");
        out.amp[((size_t)r * q + j) * 4 + k] = make_double2(a[k].real(), a[k].imag());
      }
    }
  }
  return EMS_OK;
}

#define HIPCHK(h, call)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail((h), e_ == hipErrorOutOfMemory ? EMS_ERR_OOM : EMS_ERR_HIP,            \
                  std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_));  \
  } while (0)

template <typename T>
void dfree(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void clear_prof(ems_handle *h) {
  for (auto &r : h->prof_recs) {
    if (r.a) (void)hipEventDestroy(r.a);
    if (r.b) (void)hipEventDestroy(r.b);
  }
  h->prof_recs.clear();
}

void drop_graphs(ems_handle *h) {
  for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second.first);
  h->graphs.clear();
}

void free_device(ems_handle *h) {
  drop_graphs(h);
  clear_prof(h);
  dfree(h->d_xy);
  dfree(h->d_p);
  dfree(h->d_off);
  dfree(h->d_S);
  dfree(h->d_S32);
  dfree(h->d_Soff);
  dfree(h->d_xi);
  dfree(h->d_w);
  dfree(h->d_sp);
  dfree(h->d_ss);
  dfree(h->d_R);
  dfree(h->d_dR);
  dfree(h->d_Tu);
  dfree(h->d_spb);
  dfree(h->d_ssb);
  if (h->ext) {
    ems_destroy(h->ext);
    h->ext = nullptr;
  }
  dfree(h->d_Vp);
  dfree(h->d_Vs);
  dfree(h->d_Eagg);
  dfree(h->d_Edis);
  dfree(h->d_Eagg32);
  dfree(h->d_Edis32);
  dfree(h->d_EaggA);
  dfree(h->d_EdisA);
  dfree(h->d_gco);
  dfree(h->d_xys);
  dfree(h->d_xpad);
  dfree(h->d_bpad);
  dfree(h->d_sperm);
  dfree(h->d_kcut);
  dfree(h->d_jr);
  dfree(h->d_kcut_f);
  dfree(h->d_jr_f);
  h->cut_f_depth = -1.0;
  h->depth_kept = 1.0;
  dfree(h->d_VpA_agg);
  dfree(h->d_VsA_agg);
  dfree(h->d_VpA_dis);
  dfree(h->d_VsA_dis);
  dfree(h->d_irR);
  dfree(h->d_irD);
  h->ir_bytes = 0;
  dfree(h->d_agg);
  dfree(h->d_refl);
  dfree(h->d_dis);
  dfree(h->d_free);
  dfree(h->d_V);
  dfree(h->d_tmp);
  dfree(h->d_red);
  dfree(h->d_pool);
  dfree(h->d_fmm_part);
  dfree(h->d_nsym);
  dfree(h->d_mult);
  dfree(h->d_loc);
  dfree(h->d_nbr_ptr);
  dfree(h->d_nbr_idx);
  dfree(h->d_nbr_off);
  dfree(h->d_nbr_p);
  dfree(h->d_adj1);
  dfree(h->d_adj2);
  for (auto &D : h->fmm_dev) {
    dfree(D.ptr);
    dfree(D.in_P);
    dfree(D.sym_L);
    dfree(D.sgn);
    dfree(D.out_P);
    dfree(D.item_out);
    dfree(D.item_row0);
    dfree(D.item_t0);
    dfree(D.item_t1);
    dfree(D.item_slot);
    dfree(D.red_out);
    dfree(D.red_row0);
    dfree(D.red_slot0);
    dfree(D.red_g);
    dfree(D.in_base);
    dfree(D.sym_base);
    dfree(D.out_base);
  }
  h->fmm_dev.clear();
  {
    ems::M2lDev &G = h->m2l_dev;
    dfree(G.g_P);
    dfree(G.g_G);
    dfree(G.g_nb);
    dfree(G.g_off);
    dfree(G.g_poff);
    dfree(G.tile_ptr);
    dfree(G.tile_box);
    dfree(G.ent_sym);
    dfree(G.ent_src);
    dfree(G.it_g);
    dfree(G.it_rt);
    dfree(G.it_tile);
    dfree(G.it_e0);
    dfree(G.it_e1);
    dfree(G.it_slot);
  }
  dfree(h->d_m2l_part);
  h->ws_nrhs = 0;
  h->V_bytes = h->tmp_bytes = h->red_bytes = 0;
  dfree(h->d_pc_rptr);
  dfree(h->d_pc_rows);
  dfree(h->d_pc_nb);
  dfree(h->d_pc_ioff);
  dfree(h->d_pc_inv);
  dfree(h->d_pcz);
  h->pcz_bytes = 0;
  h->pc_built = false;
  h->pc_nc = h->pc_n2 = 0;
  h->pc_store = 0;
}

template <typename T>
int upload(ems_handle *h, T *&dst, const T *src, size_t count) {
  dfree(dst);
  if (count == 0) return EMS_OK;
  HIPCHK(h, hipMalloc(&dst, count * sizeof(T)));
  HIPCHK(h, hipMemcpy(dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  return EMS_OK;
}

bool finite_all(const double *v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// Workspace for nrhs right-hand sides.
// Elements of the matrix-core aggregate's padded coefficient copy.
size_t xpad_len(const ems_handle *h, int nrhs) {
  const int nw = 16 * ((2 * ems::pm_bucket(h->pmax) + 1 + 15) / 16);
  return (size_t)nrhs * 2 * h->n * nw;
}

// ... and of the disaggregate's padded B operand.
size_t bpad_len(const ems_handle *h, int nrhs) {
  const int nw = 16 * ((2 * ems::pm_bucket(h->pmax) + 1 + 15) / 16);
  return (size_t)nrhs * 2 * h->q * nw;
}

int ensure_ws(ems_handle *h, int nrhs) {
  if (h->ws_nrhs >= nrhs) return EMS_OK;
  ++h->ws_epoch;
  dfree(h->d_agg);
  dfree(h->d_refl);
  dfree(h->d_dis);
  dfree(h->d_free);
  const int node_tiles = (h->q + 255) / 256;
  const int part_tiles = (h->n + 255) / 256;
  h->agg_chunks = std::max(1, std::min(std::max(1, h->n / 8),
                                       (4096 + 2 * nrhs * node_tiles - 1) / (2 * nrhs * node_tiles)));
  h->dis_chunks = std::max(1, std::min(std::max(1, h->q / 32),
                                       (ems::kDisChunkTarget + 2 * nrhs * part_tiles - 1) / (2 * nrhs * part_tiles)));
  const size_t nc = (size_t)h->ncoef;
  HIPCHK(h, hipMalloc(&h->d_agg, sizeof(double2) * (size_t)nrhs * 2 * h->agg_chunks * h->q));
  HIPCHK(h, hipMalloc(&h->d_refl, sizeof(double2) * (size_t)nrhs * 2 * h->q));
  HIPCHK(h, hipMalloc(&h->d_dis, sizeof(double2) * (size_t)nrhs * h->dis_chunks * nc));
  HIPCHK(h, hipMalloc(&h->d_free, sizeof(double2) * (size_t)nrhs * nc));
  dfree(h->d_xpad);
  dfree(h->d_bpad);
  if (ems::somm_mfma_ready(h, false) || ems::somm_mfma_ready(h, true)) {
    HIPCHK(h, hipMalloc(&h->d_xpad, sizeof(double2) * xpad_len(h, nrhs)));
    HIPCHK(h, hipMalloc(&h->d_bpad, sizeof(double2) * bpad_len(h, nrhs)));
  }
  dfree(h->d_mult);
  dfree(h->d_loc);
  dfree(h->d_fmm_part);
  dfree(h->d_adj1);
  dfree(h->d_adj2);
  if (h->fmm_on) {
    HIPCHK(h, hipMalloc(&h->d_mult, sizeof(double2) * (size_t)nrhs * h->fmm.exp_len));
    HIPCHK(h, hipMalloc(&h->d_loc, sizeof(double2) * (size_t)nrhs * h->fmm.exp_len));
    if (h->fmm.max_slots > 0)
      HIPCHK(h, hipMalloc(&h->d_fmm_part,
                          sizeof(double2) * (size_t)nrhs * h->fmm.max_slots * ems::kFmmRows));
    dfree(h->d_m2l_part);
    if (h->fmm.m2l.part_len > 0)
      HIPCHK(h, hipMalloc(&h->d_m2l_part, sizeof(double2) * (size_t)nrhs * h->fmm.m2l.part_len));
  }
  h->ws_nrhs = nrhs;
  return EMS_OK;
}

int ensure_tmp(ems_handle *h, size_t bytes) {
  if (h->tmp_bytes >= bytes) return EMS_OK;
  ++h->ws_epoch;
  dfree(h->d_tmp);
  HIPCHK(h, hipMalloc(&h->d_tmp, bytes));
  h->tmp_bytes = bytes;
  return EMS_OK;
}

int ensure_red(ems_handle *h, size_t bytes) {
  if (h->red_bytes >= bytes) return EMS_OK;
  dfree(h->d_red);
  HIPCHK(h, hipMalloc(&h->d_red, bytes));
  h->red_bytes = bytes;
  return EMS_OK;
}

int check_geometry(ems_handle *h) {
  const int n = h->n;
  double Rmax = 0;
  for (int i = 0; i < n; ++i) {
    if (!(h->R[i] > 0)) return fail(h, EMS_ERR_GEOMETRY, "enclosing radius must be > 0");
    if (!(h->xy[2 * i + 1] + h->R[i] < 0))
      return fail(h, EMS_ERR_GEOMETRY,
                  "particle " + std::to_string(i) + ": enclosing disk reaches the interface y = 0");
    Rmax = std::max(Rmax, h->R[i]);
  }
  // cell grid with cell >= 2 Rmax: overlapping disks are in neighbouring cells
  const double cell = 2.0 * Rmax;
  std::map<std::pair<long, long>, std::vector<int>> grid;
  for (int i = 0; i < n; ++i)
    grid[{(long)std::floor(h->xy[2 * i] / cell), (long)std::floor(h->xy[2 * i + 1] / cell)}]
        .push_back(i);
  for (int i = 0; i < n; ++i) {
    const long cx = (long)std::floor(h->xy[2 * i] / cell);
    const long cy = (long)std::floor(h->xy[2 * i + 1] / cell);
    for (long gx = cx - 1; gx <= cx + 1; ++gx)
      for (long gy = cy - 1; gy <= cy + 1; ++gy) {
        auto it = grid.find({gx, gy});
        if (it == grid.end()) continue;
        for (int j : it->second) {
          if (j <= i) continue;
          const double dx = h->xy[2 * i] - h->xy[2 * j], dy = h->xy[2 * i + 1] - h->xy[2 * j + 1];
          if (std::sqrt(dx * dx + dy * dy) <= h->R[i] + h->R[j])
            return fail(h, EMS_ERR_GEOMETRY,
                        "enclosing disks of particles " + std::to_string(i) + " and " +
                            std::to_string(j) + " overlap");
        }
      }
  }
  return EMS_OK;
}

int apply_impl(ems_handle *h, const double2 *x, double2 *y, int nrhs, int flags, bool adjoint,
               hipStream_t st) {
  const bool mixed = (flags & EMS_MIXED) != 0;
  // FP32 near field unless its Hankel symbols could overflow FP32 (build)
  const bool mixed_near = mixed && !h->near_fp64;
  const int parts = flags & 15;
  if ((parts & EMS_PART_IDENTITY) && !(parts & EMS_PART_S))
    return fail(h, EMS_ERR_ARG, "EMS_PART_IDENTITY needs EMS_PART_S");
  int rc = ensure_ws(h, nrhs);
  if (rc) return rc;
  const double2 *src = x;
  if (adjoint && (parts & EMS_PART_S)) {
    rc = ensure_tmp(h, sizeof(double2) * (size_t)nrhs * h->ncoef);
    if (rc) return rc;
    ems::ProfScope ps(h, "s_apply_adjoint", st, h->flops_s * nrhs);
    HIPCHK(h, ems::launch_s_apply(h, x, h->d_tmp, nrhs, true, st));
    src = h->d_tmp;
  }
  if (parts & EMS_PART_FREE) {
    if (!h->fmm_on) {
      ems::ProfScope ps(h, "graf_direct", st, h->flops_graf * nrhs);
      HIPCHK(h, ems::launch_graf_direct(h, src, h->d_free, nrhs, adjoint, mixed_near, st));
    } else if (!adjoint) {
      {
        ems::ProfScope ps(h, "graf_near", st, h->flops_graf * nrhs);
        HIPCHK(h, ems::launch_graf_direct(h, src, h->d_free, nrhs, false, mixed_near, st));
      }
      HIPCHK(h, ems::launch_fmm(h, src, h->d_free, nrhs, mixed, st));
    } else {
      // reciprocity: T^H v = P conj(T conj(P v))
      const size_t bytes = sizeof(double2) * (size_t)nrhs * h->ncoef;
      if (h->adj_bytes < bytes) {
        ++h->ws_epoch;
        dfree(h->d_adj1);
        dfree(h->d_adj2);
        HIPCHK(h, hipMalloc(&h->d_adj1, bytes));
        HIPCHK(h, hipMalloc(&h->d_adj2, bytes));
        h->adj_bytes = bytes;
      }
      HIPCHK(h, ems::launch_conj_flip(h, src, h->d_adj1, nrhs, st));
      {
        ems::ProfScope ps(h, "graf_near", st, h->flops_graf * nrhs);
        HIPCHK(h, ems::launch_graf_direct(h, h->d_adj1, h->d_adj2, nrhs, false, mixed_near, st));
      }
      HIPCHK(h, ems::launch_fmm(h, h->d_adj1, h->d_adj2, nrhs, mixed, st));
      HIPCHK(h, ems::launch_conj_flip(h, h->d_adj2, h->d_free, nrhs, st));
    }
  }
  if (parts & EMS_PART_REFL) {
    // one complex multiply-add per (node, coefficient) in each contraction,
    // over the (node, particle) pairs the depth truncation keeps when the
    // tabulated kernels run
    const bool tab = ems::somm_mfma_ready(h, adjoint);
    const double fc = 8.0 * (double)h->q * (double)h->ncoef * nrhs * (tab ? h->depth_kept : 1.0);
    {
      ems::ProfScope ps(h, "somm_aggregate", st, fc);
      HIPCHK(h, ems::launch_somm_aggregate(h, src, nrhs, adjoint, mixed, st));
    }
    {
      ems::ProfScope ps(h, "somm_reflect", st);
      HIPCHK(h, ems::launch_somm_reflect(h, nrhs, adjoint, st));
    }
    {
      ems::ProfScope ps(h, "somm_disaggregate", st, fc);
      HIPCHK(h, ems::launch_somm_disaggregate(h, nrhs, adjoint, mixed, st));
    }
  }
  int cflags = parts;
  if (adjoint) cflags &= ~EMS_PART_S;
  ems::ProfScope ps(h, "combine_s_apply", st, (cflags & EMS_PART_S) ? h->flops_s * nrhs : 0.0);
  HIPCHK(h, ems::launch_combine(h, x, y, nrhs, cflags, adjoint, mixed, st));
  return EMS_OK;
}

// Clusters of the block-Jacobi preconditioner: recursive splits of the
// particle set across the wider extent of its bounding box, the left part
// taking as many whole clusters of cap unknowns as half of the clusters the
// set needs, until a set fits in cap unknowns.  order receives the particles
// cluster by cluster, cptr[c] the start of cluster c in order.
void kd_clusters(const ems_handle *h, int64_t cap, std::vector<int> &order,
                 std::vector<int> &cptr) {
  const int n = h->n;
  order.resize(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  cptr.assign(1, 0);
  auto K = [&](int i) { return h->off[i + 1] - h->off[i]; };
  std::function<void(int, int)> rec = [&](int lo, int hi) {
    int64_t tot = 0;
    double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
    for (int k = lo; k < hi; ++k) {
      const int i = order[k];
      tot += K(i);
      x0 = std::min(x0, h->xy[2 * i]);
      x1 = std::max(x1, h->xy[2 * i]);
      y0 = std::min(y0, h->xy[2 * i + 1]);
      y1 = std::max(y1, h->xy[2 * i + 1]);
    }
    if (tot <= cap || hi - lo == 1) {
      cptr.push_back(hi);
      return;
    }
    const int ax = (x1 - x0) >= (y1 - y0) ? 0 : 1;
    std::sort(order.begin() + lo, order.begin() + hi, [&](int a, int b) {
      const double va = h->xy[2 * a + ax], vb = h->xy[2 * b + ax];
      return va < vb || (va == vb && a < b);
    });
    const int64_t ncl = (tot + cap - 1) / cap;
    const int64_t target = cap * ((ncl + 1) / 2);
    int sp = lo;
    int64_t acc = 0;
    while (sp < hi - 1 && acc + K(order[sp]) <= target) acc += K(order[sp++]);
    if (sp == lo) sp = lo + 1;
    rec(lo, sp);
    rec(sp, hi);
  };
  rec(0, n);
}

// Build the cluster block-Jacobi preconditioner (once per build).
int build_precond(ems_handle *h, hipStream_t st) {
  if (h->pc_built) return EMS_OK;
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<int> order, cptr;
  kd_clusters(h, h->pc_cap, order, cptr);
  const int nc = (int)cptr.size() - 1;
  std::vector<int> rptr(nc + 1, 0), rows, nb(nc);
  std::vector<int64_t> ioff(nc + 1, 0);
  rows.reserve((size_t)h->ncoef);
  int bmax = 0;
  for (int c = 0; c < nc; ++c) {
    for (int k = cptr[c]; k < cptr[c + 1]; ++k) {
      const int m = order[k];
      for (int64_t g = h->off[m]; g < h->off[m + 1]; ++g) rows.push_back((int)g);
    }
    rptr[c + 1] = (int)rows.size();
    nb[c] = rptr[c + 1] - rptr[c];
    bmax = std::max(bmax, nb[c]);
    ioff[c + 1] = ioff[c] + (int64_t)nb[c] * nb[c];
  }
  const int n2 = (bmax + 15) / 16 * 16;
  if (n2 > 512) return fail(h, EMS_ERR_ARG, "a particle block exceeds the cluster size limit");
  int rc;
  if ((rc = upload(h, h->d_pc_rptr, rptr.data(), rptr.size()))) return rc;
  if ((rc = upload(h, h->d_pc_rows, rows.data(), rows.size()))) return rc;
  if ((rc = upload(h, h->d_pc_nb, nb.data(), nb.size()))) return rc;
  if ((rc = upload(h, h->d_pc_ioff, ioff.data(), ioff.size()))) return rc;
  dfree(h->d_pc_inv);
  HIPCHK(h, hipMalloc(&h->d_pc_inv, sizeof(float2) * (size_t)std::max<int64_t>(1, ioff[nc])));
  // working matrices [B_c | I] in batches
  const int64_t mstride = (int64_t)n2 * 2 * n2;
  const size_t mbytes = sizeof(double2) * (size_t)mstride;
  size_t fr = 0, tot = 0;
  HIPCHK(h, hipMemGetInfo(&fr, &tot));
  const size_t budget = std::min<size_t>((size_t)4 << 30, (size_t)(0.3 * (double)fr));
  const int bcnt = (int)std::max<size_t>(1, std::min<size_t>((size_t)nc, budget / mbytes));
  double2 *W = nullptr;
  int *info = nullptr, *dpairs = nullptr;
  std::vector<int> pairs, hinfo(bcnt);
  int rcode = EMS_OK;
  auto cleanup = [&]() {
    dfree(W);
    dfree(info);
    dfree(dpairs);
  };
  size_t pairs_cap = 0;
  if (hipMalloc(&W, mbytes * bcnt) != hipSuccess || hipMalloc(&info, sizeof(int) * bcnt) != hipSuccess) {
    cleanup();
    return fail(h, EMS_ERR_OOM, "no device memory for the preconditioner's working matrices");
  }
  for (int c0 = 0; c0 < nc && rcode == EMS_OK; c0 += bcnt) {
    const int cnt = std::min(bcnt, nc - c0);
    pairs.clear();
    for (int c = c0; c < c0 + cnt; ++c) {
      int ro = 0;
      for (int a = cptr[c]; a < cptr[c + 1]; ++a) {
        const int m = order[a];
        int co = 0;
        for (int b = cptr[c]; b < cptr[c + 1]; ++b) {
          const int l = order[b];
          if (l != m) {
            pairs.push_back(c - c0);
            pairs.push_back(m);
            pairs.push_back(l);
            pairs.push_back(ro);
            pairs.push_back(co);
          }
          co += (int)(h->off[l + 1] - h->off[l]);
        }
        ro += (int)(h->off[m + 1] - h->off[m]);
      }
    }
    if (pairs.size() > pairs_cap) {
      dfree(dpairs);
      pairs_cap = pairs.size();
      if (hipMalloc(&dpairs, sizeof(int) * pairs_cap) != hipSuccess) {
        rcode = fail(h, EMS_ERR_OOM, "no device memory for the cluster pair list");
        break;
      }
    }
    hipError_t e = hipMemsetAsync(info, 0, sizeof(int) * cnt, st);
    if (e == hipSuccess && !pairs.empty())
      e = hipMemcpyAsync(dpairs, pairs.data(), sizeof(int) * pairs.size(), hipMemcpyHostToDevice, st);
    ems::PcBatch bt;
    bt.c0 = c0;
    bt.cnt = cnt;
    bt.pairs = dpairs;
    bt.npairs = (int)(pairs.size() / 5);
    if (e == hipSuccess) e = ems::launch_pc_factor_batch(h, bt, W, n2, mstride, info, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hinfo.data(), info, sizeof(int) * cnt, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      rcode = fail(h, EMS_ERR_HIP, std::string("preconditioner set-up: ") + hipGetErrorString(e));
      break;
    }
    for (int i = 0; i < cnt; ++i)
      if (hinfo[i]) rcode = fail(h, EMS_ERR_NUMERIC, "singular cluster block in the preconditioner");
  }
  cleanup();
  if (rcode != EMS_OK) return rcode;
  h->pc_nc = nc;
  h->pc_n2 = n2;
  h->pc_bmax = bmax;
  h->pc_store = ioff[nc];
  h->pc_built = true;
  h->pc_setup_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return EMS_OK;
}

int ensure_pcz(ems_handle *h, int nrhs) {
  const size_t bytes = sizeof(double2) * 2 * (size_t)nrhs * h->ncoef;
  if (h->pcz_bytes >= bytes) return EMS_OK;
  dfree(h->d_pcz);
  h->pcz_bytes = 0;
  HIPCHK(h, hipMalloc(&h->d_pcz, bytes));
  h->pcz_bytes = bytes;
  return EMS_OK;
}

}  // namespace

extern "C" {

int ems_create(ems_handle **out) {
  if (!out) return EMS_ERR_ARG;
  ems_handle *h = new (std::nothrow) ems_handle();
  if (!h) return EMS_ERR_OOM;
  // No device is touched before ems_build, so argument and geometry checks
  // also run on hosts without a GPU.
  if (hipGetDevice(&h->device) != hipSuccess) h->device = -1;
  *out = h;
  return EMS_OK;
}

void ems_destroy(ems_handle *h) {
  if (!h) return;
  free_device(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (auto &e : h->cap_ev)
    if (e) (void)hipEventDestroy(e);
  delete h;
}

const char *ems_last_error(const ems_handle *h) { return h ? h->err.c_str() : "null handle"; }

int ems_profile(ems_handle *h, int32_t enable) {
  if (!h) return EMS_ERR_ARG;
  if (enable) clear_prof(h);
  h->prof = enable != 0;
  return EMS_OK;
}

int ems_profile_read(ems_handle *h, ems_kernel_time *out, int32_t cap, int32_t *count) {
  if (!h || !count || (cap > 0 && !out)) return EMS_ERR_ARG;
  std::vector<std::string> names;
  std::vector<int> launches;
  std::vector<double> ms, fl;
  for (auto &r : h->prof_recs) {
    HIPCHK(h, hipEventSynchronize(r.b));
    float t = 0.f;
    HIPCHK(h, hipEventElapsedTime(&t, r.a, r.b));
    size_t k = 0;
    for (; k < names.size(); ++k)
      if (names[k] == r.name) break;
    if (k == names.size()) {
      names.push_back(r.name);
      launches.push_back(0);
      ms.push_back(0.0);
      fl.push_back(0.0);
    }
    launches[k] += 1;
    ms[k] += t;
    fl[k] += r.flops;
  }
  *count = (int32_t)names.size();
  for (int k = 0; k < (int)names.size() && k < cap; ++k) {
    std::memset(out[k].name, 0, sizeof(out[k].name));
    std::strncpy(out[k].name, names[k].c_str(), sizeof(out[k].name) - 1);
    out[k].launches = launches[k];
    out[k].total_ms = ms[k];
    out[k].flops = fl[k];
  }
  return EMS_OK;
}

int ems_set_media(ems_handle *h, const ems_media *m) {
  if (!h || !m) return EMS_ERR_ARG;
  const double v[7] = {m->host.lambda, m->host.mu, m->host.rho, m->substrate.lambda,
                       m->substrate.mu, m->substrate.rho, m->omega};
  if (!finite_all(v, 7)) return fail(h, EMS_ERR_NUMERIC, "non-finite media parameter");
  if (!(m->host.mu > 0 && m->host.lambda + m->host.mu > 0 && m->substrate.mu > 0 &&
        m->substrate.lambda + m->substrate.mu > 0 && m->host.rho > 0 && m->substrate.rho > 0 &&
        m->omega > 0))
    return fail(h, EMS_ERR_ARG, "need mu > 0, lambda + mu > 0, rho > 0, omega > 0");
  h->md = ems::make_media(*m);
  h->have_media = true;
  h->built = false;
  return EMS_OK;
}

int ems_set_particles(ems_handle *h, int32_t n, const double *xy, const double *R,
                      const int32_t *p) {
  if (!h) return EMS_ERR_ARG;
  // any failure leaves the handle without particles: nothing set before
  // survives a rejected call
  h->have_particles = false;
  h->have_s = false;
  h->built = false;
  if (n <= 0 || !xy || !R || !p) return fail(h, EMS_ERR_ARG, "bad particle arguments");
  if (!finite_all(xy, 2 * (size_t)n) || !finite_all(R, n))
    return fail(h, EMS_ERR_NUMERIC, "non-finite particle data");
  std::vector<int64_t> off(n + 1, 0);
  int pmax = 0;
  for (int i = 0; i < n; ++i) {
    if (p[i] < 1 || p[i] > ems::kMaxP)
      return fail(h, EMS_ERR_UNIMPLEMENTED, "truncation order must be in [1, 16]");
    if (!(R[i] > 0)) return fail(h, EMS_ERR_ARG, "enclosing radii must be positive");
    off[i + 1] = off[i] + 2 * (2 * p[i] + 1);
    pmax = std::max(pmax, p[i]);
  }
  h->n = n;
  h->xy.assign(xy, xy + 2 * (size_t)n);
  h->R.assign(R, R + n);
  h->p.assign(p, p + n);
  h->off = std::move(off);
  h->pmax = pmax;
  h->ncoef = h->off[n];
  h->have_particles = true;
  return EMS_OK;
}

int ems_set_smatrices(ems_handle *h, const double *S, const int64_t *offsets) {
  if (!h) return EMS_ERR_ARG;
  h->have_s = false;
  h->built = false;
  if (!S || !offsets) return fail(h, EMS_ERR_ARG, "null S");
  if (!h->have_particles) return fail(h, EMS_ERR_STATE, "set particles before S-matrices");
  if (offsets[0] != 0) return fail(h, EMS_ERR_ARG, "S offsets must start at 0");
  for (int i = 0; i < h->n; ++i) {
    const int64_t K = 4 * h->p[i] + 2;
    if (offsets[i + 1] - offsets[i] != K * K)
      return fail(h, EMS_ERR_ARG, "S offsets do not match (4p+2)^2 blocks");
  }
  h->S_off.assign(offsets, offsets + h->n + 1);
  const size_t tot = (size_t)offsets[h->n];
  if (!finite_all(S, 2 * tot)) return fail(h, EMS_ERR_NUMERIC, "non-finite S entry");
  h->S_host.resize(tot);
  for (size_t k = 0; k < tot; ++k) h->S_host[k] = cd(S[2 * k], S[2 * k + 1]);
  h->have_s = true;
  h->built = false;
  return EMS_OK;
}

int ems_set_smatrices_rotated(ems_handle *h, int32_t nproto, const double *S_proto,
                              const int64_t *proto_off, const int32_t *which,
                              const double *theta0) {
  if (!h) return EMS_ERR_ARG;
  h->have_s = false;
  h->built = false;
  if (nproto <= 0 || !S_proto || !proto_off || !which || !theta0)
    return fail(h, EMS_ERR_ARG, "bad prototype arguments");
  if (!h->have_particles) return fail(h, EMS_ERR_STATE, "set particles before S-matrices");
  for (int k = 0; k < nproto; ++k)
    if (proto_off[k + 1] < proto_off[k] || proto_off[0] != 0)
      return fail(h, EMS_ERR_ARG, "prototype offsets must increase from 0");
  if (!finite_all(S_proto, 2 * (size_t)proto_off[nproto]))
    return fail(h, EMS_ERR_NUMERIC, "non-finite prototype entry");
  std::vector<int64_t> soff(h->n + 1, 0);
  for (int i = 0; i < h->n; ++i) {
    const int64_t K = 4 * h->p[i] + 2;
    if (which[i] < 0 || which[i] >= nproto)
      return fail(h, EMS_ERR_ARG, "prototype index out of range");
    if (proto_off[which[i] + 1] - proto_off[which[i]] != K * K)
      return fail(h, EMS_ERR_ARG, "prototype size does not match the particle's (4p+2)^2");
    if (!std::isfinite(theta0[i])) return fail(h, EMS_ERR_NUMERIC, "non-finite orientation");
    soff[i + 1] = soff[i] + K * K;
  }
  // S_m = D S D^H, D = diag(e^{-i n theta}) over [alpha_{-p..p}, beta_{-p..p}]
  h->S_host.resize((size_t)soff[h->n]);
  std::vector<cd> d;
  for (int i = 0; i < h->n; ++i) {
    const int pm = h->p[i], N = 2 * pm + 1, K = 2 * N;
    d.resize(K);
    for (int r = 0; r < K; ++r) d[r] = std::polar(1.0, -(double)((r % N) - pm) * theta0[i]);
    const double *src = S_proto + 2 * proto_off[which[i]];
    cd *dst = h->S_host.data() + soff[i];
    for (int r = 0; r < K; ++r)
      for (int c = 0; c < K; ++c) {
        const size_t e = (size_t)r * K + c;
        dst[e] = d[r] * cd(src[2 * e], src[2 * e + 1]) * std::conj(d[c]);
      }
  }
  h->S_off = soff;
  h->have_s = true;
  h->built = false;
  return EMS_OK;
}

int ems_smatrix_disk(const ems_media *m, double a, int32_t p, int32_t bc, double *S_out) {
  if (!m || !S_out || !(a > 0) || p < 0 || (bc != 0 && bc != 1)) return EMS_ERR_ARG;
  std::vector<cd> S;
  const int rc = ems::disk_smatrix(ems::make_media(*m), a, p, bc, S);
  if (rc) return rc;
  for (size_t k = 0; k < S.size(); ++k) {
    S_out[2 * k] = S[k].real();
    S_out[2 * k + 1] = S[k].imag();
  }
  return EMS_OK;
}

namespace {
// Device buffers of one ems_smatrix_shapes call, freed on every return path.
struct ShapeBufs {
  std::vector<void *> ptrs;
  ~ShapeBufs() {
    for (void *q : ptrs) (void)hipFree(q);
  }
  hipError_t get(void **out, size_t bytes) {
    *out = nullptr;
    const hipError_t e = hipMalloc(out, bytes);
    if (e == hipSuccess) ptrs.push_back(*out);
    return e;
  }
};
}  // namespace

int ems_smatrix_shapes(ems_handle *h, const int32_t *kind, const double *a, const double *theta0,
                       const int32_t *bc, int32_t npts, double delta, void *S_out,
                       ems_stream_t stream) {
  if (!h || !kind || !a || !theta0 || !bc || !S_out)
    return fail(h, EMS_ERR_ARG, "bad shape arguments");
  if (!h->have_media || !h->have_particles)
    return fail(h, EMS_ERR_STATE, "set media and particles before generating S-matrices");
  const int N = npts == 0 ? 256 : npts;
  if (N < 16 || N > 256 || N % 8 != 0)
    return fail(h, EMS_ERR_ARG, "npts must be a multiple of 8 in [16, 256]");
  if (!std::isfinite(delta)) return fail(h, EMS_ERR_ARG, "non-finite delta");
  const int n = h->n;
  static const double kDelta[5] = {0.3, 0.2, 0.12, 0.2, 0.16};
  static const double kExtent[5] = {1.0, 1.0, 1.3, 1.25, 1.25};   // max |z(t)| / a
  std::vector<int> hk(n), hbc(n);
  std::vector<double> ha(n), hct(n), hst(n), hdl(n);
  std::vector<int64_t> soff(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    if (kind[i] < 0 || kind[i] > 4) return fail(h, EMS_ERR_ARG, "shape kind must be 0 .. 4");
    if (bc[i] != 0 && bc[i] != 1) return fail(h, EMS_ERR_ARG, "bc must be 0 or 1");
    if (!(a[i] > 0) || !std::isfinite(a[i]) || !std::isfinite(theta0[i]))
      return fail(h, EMS_ERR_ARG, "shape size must be positive and finite");
    if (a[i] * kExtent[kind[i]] > h->R[i] * (1.0 + 1e-12))
      return fail(h, EMS_ERR_GEOMETRY, "shape leaves its enclosing disk");
    hk[i] = kind[i];
    hbc[i] = bc[i];
    ha[i] = a[i];
    hct[i] = std::cos(theta0[i]);
    hst[i] = std::sin(theta0[i]);
    hdl[i] = delta > 0 ? delta : kDelta[kind[i]];
    const int64_t K = 4 * h->p[i] + 2;
    soff[i + 1] = soff[i] + K * K;
  }
  hipStream_t st = (hipStream_t)stream;
  const int n2 = 2 * N, nrmax = 2 * (2 * h->pmax + 1);
  const int64_t mstride = (int64_t)n2 * (n2 + nrmax), estride = (int64_t)nrmax * N;
  const int64_t per = (int64_t)sizeof(double2) * (mstride + estride);
  // workspace batch: at most 6 GiB and 40 % of the free device memory
  size_t fre = 0, tot = 0;
  (void)hipMemGetInfo(&fre, &tot);
  const int64_t cap = std::min<int64_t>((int64_t)6 << 30, (int64_t)(0.4 * (double)fre));
  const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(n, cap / per));
  ShapeBufs B;
  void *d_i = nullptr, *d_d = nullptr, *d_off = nullptr, *d_W = nullptr, *d_E = nullptr,
       *d_info = nullptr;
  HIPCHK(h, B.get(&d_i, sizeof(int) * 3 * (size_t)n));
  HIPCHK(h, B.get(&d_d, sizeof(double) * 4 * (size_t)n));
  HIPCHK(h, B.get(&d_off, sizeof(int64_t) * (size_t)(n + 1)));
  HIPCHK(h, B.get(&d_W, sizeof(double2) * (size_t)mstride * chunk));
  HIPCHK(h, B.get(&d_E, sizeof(double2) * (size_t)estride * chunk));
  HIPCHK(h, B.get(&d_info, sizeof(int) * (size_t)chunk));
  int *di = (int *)d_i;
  double *dd = (double *)d_d;
  HIPCHK(h, hipMemcpyAsync(di, hk.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(di + n, h->p.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(di + 2 * n, hbc.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(dd, ha.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(dd + n, hct.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(dd + 2 * n, hst.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(dd + 3 * n, hdl.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(d_off, soff.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice,
                           st));
  const ems::MfsBatch mb{&h->md, N, di, di + n, di + 2 * n, dd, dd + n, dd + 2 * n, dd + 3 * n,
                         (const int64_t *)d_off};
  std::vector<int> info(chunk);
  for (int i0 = 0; i0 < n; i0 += chunk) {
    const int cnt = std::min(chunk, n - i0);
    HIPCHK(h, hipMemsetAsync(d_info, 0, sizeof(int) * cnt, st));
    HIPCHK(h, ems::launch_mfs_smatrices(mb, i0, cnt, (double2 *)d_W, mstride, (double2 *)d_E,
                                         estride, (int *)d_info, (double2 *)S_out, st));
    HIPCHK(h, hipMemcpyAsync(info.data(), d_info, sizeof(int) * cnt, hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    for (int c = 0; c < cnt; ++c)
      if (info[c]) return fail(h, EMS_ERR_NUMERIC, "singular collocation system of a particle");
  }
  return EMS_OK;
}

static int spec_from(const ems_sommerfeld *s, ems::SommerfeldSpec &o, std::string &err) {
  if (s->kind < 0 || s->kind > 3) {
    err = "sommerfeld kind must be 0, 1, 2, 3";
    return EMS_ERR_ARG;
  }
  o.kind = s->kind;
  o.q = s->q;
  o.t_max = s->t_max;
  o.delta = s->delta > 0 ? s->delta : 0.5;
  o.panel_scale = s->panel_scale > 0 ? s->panel_scale : 1.0;
  o.panel_order = s->panel_order > 0 ? s->panel_order : 64;
  o.tail_factor = s->tail_factor > 0 ? s->tail_factor : 1.0;
  o.depth_cut = s->depth_cut > 0 ? s->depth_cut : (s->depth_cut < 0 ? 0.0 : 1e-26);
  if (o.panel_order < 8 || o.panel_order > 256) {
    err = "panel_order must be in [8, 256]";
    return EMS_ERR_ARG;
  }
  o.user.clear();
  if (s->kind == 2) {
    if (!s->nodes || s->q <= 0) {
      err = "kind 2 needs q nodes";
      return EMS_ERR_ARG;
    }
    o.user.assign(s->nodes, s->nodes + 4 * (size_t)s->q);
  }
  return EMS_OK;
}

int ems_sommerfeld_nodes(const ems_media *m, const ems_sommerfeld *s, int32_t n,
                         const double *xy, const int32_t *p, int32_t *q, double *nodes_out,
                         double *t_max) {
  if (!m || !s || n <= 0 || !xy || !p || !q) return EMS_ERR_ARG;
  ems::SommerfeldSpec spec;
  std::string err;
  int rc = spec_from(s, spec, err);
  if (rc) return rc;
  std::vector<double> vxy(xy, xy + 2 * (size_t)n);
  std::vector<int> vp(p, p + n);
  ems::NodeTable nt;
  rc = ems::build_nodes(spec, ems::make_media(*m), vxy, vp, nt, err);
  if (rc) return rc;
  const int cap = *q;
  *q = (int32_t)nt.xi.size();
  if (t_max) *t_max = nt.t_max;
  if (nodes_out) {
    if (cap < (int)nt.xi.size()) return EMS_ERR_ARG;
    for (size_t j = 0; j < nt.xi.size(); ++j) {
      nodes_out[6 * j] = nt.xi[j].real();
      nodes_out[6 * j + 1] = nt.xi[j].imag();
      nodes_out[6 * j + 2] = nt.w[j].real();
      nodes_out[6 * j + 3] = nt.w[j].imag();
      nodes_out[6 * j + 4] = nt.bp[j];
      nodes_out[6 * j + 5] = nt.d[j];
    }
  }
  return EMS_OK;
}

int ems_sommerfeld_depth_cuts(const ems_media *m, const ems_sommerfeld *s, int32_t n,
                              const double *xy, const int32_t *p, int32_t q, int32_t *perm_out,
                              int32_t *kcut_out, int32_t *range_out, double *kept_out) {
  if (!m || !s || n <= 0 || !xy || !p || !perm_out || !kcut_out || !range_out)
    return EMS_ERR_ARG;
  ems::SommerfeldSpec spec;
  std::string err;
  int rc = spec_from(s, spec, err);
  if (rc) return rc;
  std::vector<double> vxy(xy, xy + 2 * (size_t)n);
  std::vector<int> vp(p, p + n);
  int pmax = 0;
  for (int i = 0; i < n; ++i) pmax = std::max(pmax, vp[i]);
  ems::NodeTable nt;
  const ems::Media md = ems::make_media(*m);
  rc = ems::build_nodes(spec, md, vxy, vp, nt, err);
  if (rc) return rc;
  if (q != (int32_t)nt.xi.size()) return EMS_ERR_ARG;
  ems::DepthCuts dc;
  ems::depth_cuts(nt, md, vxy, pmax, spec.depth_cut, HUGE_VAL, dc);
  std::copy(dc.perm.begin(), dc.perm.end(), perm_out);
  std::copy(dc.kcut.begin(), dc.kcut.end(), kcut_out);
  std::copy(dc.jr.begin(), dc.jr.end(), range_out);
  if (kept_out) *kept_out = dc.kept;
  return EMS_OK;
}

int ems_reflection(const ems_media *m, double xi_re, double xi_im, double *R_out) {
  if (!m || !R_out) return EMS_ERR_ARG;
  cd R[4];
  const int rc = ems::reflection(cd(xi_re, xi_im), ems::make_media(*m), R);
  if (rc) return rc;
  for (int k = 0; k < 4; ++k) {
    R_out[2 * k] = R[k].real();
    R_out[2 * k + 1] = R[k].imag();
  }
  return EMS_OK;
}

int ems_set_sommerfeld(ems_handle *h, const ems_sommerfeld *s) {
  if (!h || !s) return EMS_ERR_ARG;
  const int rc = spec_from(s, h->somm, h->err);
  if (rc) return rc;
  h->built = false;
  return EMS_OK;
}

int ems_set_fmm(ems_handle *h, const ems_fmm *f) {
  if (!h || !f) return EMS_ERR_ARG;
  if (f->mode < 0 || f->mode > 2) return fail(h, EMS_ERR_ARG, "fmm mode must be 0, 1 or 2");
  if (f->leaf < 0 || f->top_boxes < 0 || f->digits < 0 || f->digits > 15.5)
    return fail(h, EMS_ERR_ARG, "bad fmm parameters");
  h->fmm_mode = f->mode;
  h->fmm_leaf = f->leaf > 0 ? f->leaf : 6;
  h->fmm_top = f->top_boxes > 0 ? f->top_boxes : 64;
  h->fmm_digits = f->digits > 0 ? f->digits : 13.0;
  h->built = false;
  return EMS_OK;
}

int ems_build(ems_handle *h, ems_stream_t stream) {
  (void)stream;
  if (!h) return EMS_ERR_ARG;
  if (!h->have_media || !h->have_particles || !h->have_s)
    return fail(h, EMS_ERR_STATE, "set media, particles and S-matrices before build");
  for (int i = 0; i < h->n; ++i)
    if (h->p[i] < 1 || h->p[i] > ems::kMaxP || h->p[i] > h->pmax)
      return fail(h, EMS_ERR_STATE, "particle orders outside [1, 16]");
  int rc = check_geometry(h);
  if (rc) return rc;
  free_device(h);
  // node table and per-node reflection
  ems::NodeTable nt;
  rc = ems::build_nodes(h->somm, h->md, h->xy, h->p, nt, h->err);
  if (rc) return rc;
  h->nodes = nt;
  h->q = (int)nt.xi.size();
  // power tables padded to the kernels' compile-time order (zeros beyond pmax)
  const int pmb = ems::pm_bucket(h->pmax);
  const int q = h->q, ld = 2 * pmb + 1;
  std::vector<double2> xi(q), w(q), sp(q), ss(q), spb(q), ssb(q), R(4 * (size_t)q),
      Tu(4 * (size_t)q), dR(8 * (size_t)q), Vp((size_t)q * ld), Vs((size_t)q * ld);
  const cd I(0.0, 1.0);
  double vmax = 0.0;
  for (int j = 0; j < q; ++j) {
    const cd x = nt.xi[j];
    cd s4[4];
    ems::node_s(x, nt.bp[j], nt.d[j], h->md, s4);
    const cd s1 = s4[0], s2 = s4[1];
    cd Rj[4], dRj[8], Rt[4], Tj[4];
    rc = ems::reflection_deriv_s(x, s4, h->md, Rj, dRj);
    if (rc) return fail(h, rc, "singular interface system at a Sommerfeld node");
    rc = ems::reflect_transmit_s(x, s4, h->md, Rt, Tj);
    if (rc) return fail(h, rc, "singular interface system at a Sommerfeld node");
    for (int k = 0; k < 4; ++k) Tu[4 * (size_t)j + k] = make_double2(Tj[k].real(), Tj[k].imag());
    spb[j] = make_double2(s4[2].real(), s4[2].imag());
    ssb[j] = make_double2(s4[3].real(), s4[3].imag());
    for (int k = 0; k < 8; ++k) dR[8 * (size_t)j + k] = make_double2(dRj[k].real(), dRj[k].imag());
    xi[j] = make_double2(x.real(), x.imag());
    w[j] = make_double2(nt.w[j].real(), nt.w[j].imag());
    sp[j] = make_double2(s1.real(), s1.imag());
    ss[j] = make_double2(s2.real(), s2.imag());
    for (int k = 0; k < 4; ++k) R[4 * (size_t)j + k] = make_double2(Rj[k].real(), Rj[k].imag());
    // V[j][n] = (-i zeta)^n, zeta = (xi - s)/k
    const cd zp = -I * (x - s1) / h->md.kp, zs = -I * (x - s2) / h->md.ks;
    cd ap = 1.0, as = 1.0, bp = 1.0, bs = 1.0;
    const cd izp = 1.0 / zp, izs = 1.0 / zs;
    Vp[(size_t)j * ld + pmb] = make_double2(1.0, 0.0);
    Vs[(size_t)j * ld + pmb] = make_double2(1.0, 0.0);
    for (int n = 1; n <= h->pmax; ++n) {
      ap *= zp;
      as *= zs;
      bp *= izp;
      bs *= izs;
      Vp[(size_t)j * ld + pmb + n] = make_double2(ap.real(), ap.imag());
      Vs[(size_t)j * ld + pmb + n] = make_double2(as.real(), as.imag());
      Vp[(size_t)j * ld + pmb - n] = make_double2(bp.real(), bp.imag());
      Vs[(size_t)j * ld + pmb - n] = make_double2(bs.real(), bs.imag());
    }
    vmax = std::max({vmax, std::abs(ap), std::abs(as), std::abs(bp), std::abs(bs)});
  }
  // the FP32 contractions of the mixed form carry these powers in FP32: beyond
  // 1e30 (low frequency, high order, long tails) they run in FP64 instead
  h->somm_fp64 = !(vmax < 1e30);
  // packed S store: per particle column-major
  std::vector<double2> St(h->S_host.size());
  for (int m = 0; m < h->n; ++m) {
    const int64_t K = 4 * h->p[m] + 2, o = h->S_off[m];
    for (int64_t r = 0; r < K; ++r)
      for (int64_t c = 0; c < K; ++c) {
        const cd v = h->S_host[o + r * K + c];
        St[o + c * K + r] = make_double2(v.real(), v.imag());
      }
  }
  std::vector<float2> St32(St.size());
  for (size_t k = 0; k < St.size(); ++k) St32[k] = make_float2((float)St[k].x, (float)St[k].y);
  // free-space part: direct sum or FMM (host plan, bounds-checked)
  h->fmm_on = h->fmm_mode == 2 || (h->fmm_mode == 0 && h->n > 1500);
  h->n_pairs = (int64_t)h->n * (h->n - 1);
  {
    // algorithmic work: per ordered pair both wave types, (2p_m+1)(2p_l+1)
    // complex multiply-adds each; S blocks (4p+2)^2 each
    double s1 = 0.0, s2 = 0.0;
    h->flops_s = 0.0;
    for (int m = 0; m < h->n; ++m) {
      const double k = 2.0 * h->p[m] + 1.0;
      s1 += k;
      s2 += k * k;
      h->flops_s += 8.0 * (2.0 * k) * (2.0 * k);
    }
    h->flops_graf = 16.0 * (s1 * s1 - s2);
  }
  if (h->fmm_on) {
    rc = ems::build_fmm(h, h->fmm, h->err);
    if (rc) return rc;
    h->n_pairs = (int64_t)h->fmm.nbr_idx.size();
    double f = 0.0;
    for (int m = 0; m < h->n; ++m)
      for (int t = h->fmm.nbr_ptr[m]; t < h->fmm.nbr_ptr[m + 1]; ++t)
        f += 16.0 * (2.0 * h->p[m] + 1.0) * (2.0 * h->p[h->fmm.nbr_idx[t]] + 1.0);
    h->flops_graf = f;
  }
  {
    // The mixed form runs the direct / near-field Graf sums in FP32.  Their
    // symbols H_nu(k d), |nu| <= 2 pmax, grow like (nu - 1)! (2 / k d)^nu for
    // small k d; where that passes 1e30 over the pairs the kernel visits (kp d
    // smallest), FP32 would overflow and the near field stays FP64.
    double dmin = 1e300;
    auto dist = [&](int a, int b) {
      return std::hypot(h->xy[2 * a] - h->xy[2 * b], h->xy[2 * a + 1] - h->xy[2 * b + 1]);
    };
    if (h->fmm_on) {
      for (int m = 0; m < h->n; ++m)
        for (int t = h->fmm.nbr_ptr[m]; t < h->fmm.nbr_ptr[m + 1]; ++t)
          dmin = std::min(dmin, dist(m, h->fmm.nbr_idx[t]));
    } else {
      for (int m = 0; m < h->n; ++m)
        for (int l = m + 1; l < h->n; ++l) dmin = std::min(dmin, dist(m, l));
    }
    h->near_fp64 = false;
    if (h->n > 1) {
      const double x = h->md.kp * dmin;
      double ym = std::cyl_neumann(0.0, x), y1 = std::cyl_neumann(1.0, x);
      double ymax = std::max(std::fabs(ym), std::fabs(y1));
      for (int nu = 1; nu < 2 * h->pmax && ymax < 1e30; ++nu) {
        const double yn = 2.0 * nu / x * y1 - ym;
        ym = y1;
        y1 = yn;
        ymax = std::max(ymax, std::fabs(yn));
      }
      h->near_fp64 = !(ymax < 1e30);
    }
  }
  if (h->device < 0) return fail(h, EMS_ERR_HIP, "no HIP device (host set-up completed)");
  if ((rc = upload(h, h->d_xy, h->xy.data(), h->xy.size()))) return rc;
  std::vector<int> pv(h->p.begin(), h->p.end());
  if ((rc = upload(h, h->d_p, pv.data(), pv.size()))) return rc;
  if ((rc = upload(h, h->d_off, h->off.data(), h->off.size()))) return rc;
  if ((rc = upload(h, h->d_Soff, h->S_off.data(), h->S_off.size()))) return rc;
  if ((rc = upload(h, h->d_S, St.data(), St.size()))) return rc;
  if ((rc = upload(h, h->d_S32, St32.data(), St32.size()))) return rc;
  if ((rc = upload(h, h->d_xi, xi.data(), xi.size()))) return rc;
  if ((rc = upload(h, h->d_w, w.data(), w.size()))) return rc;
  if ((rc = upload(h, h->d_sp, sp.data(), sp.size()))) return rc;
  if ((rc = upload(h, h->d_ss, ss.data(), ss.size()))) return rc;
  if ((rc = upload(h, h->d_R, R.data(), R.size()))) return rc;
  if ((rc = upload(h, h->d_dR, dR.data(), dR.size()))) return rc;
  if ((rc = upload(h, h->d_Tu, Tu.data(), Tu.size()))) return rc;
  if ((rc = upload(h, h->d_spb, spb.data(), spb.size()))) return rc;
  if ((rc = upload(h, h->d_ssb, ssb.data(), ssb.size()))) return rc;
  if ((rc = upload(h, h->d_Vp, Vp.data(), Vp.size()))) return rc;
  if ((rc = upload(h, h->d_Vs, Vs.data(), Vs.size()))) return rc;
  {
    // power tables of the adjoint matrix-core contractions: conj(V) (-1)^n
    // (aggregate of the conjugated disaggregate factors) and conj(V)
    std::vector<double2> a1(Vp.size()), a2(Vs.size()), d1(Vp.size()), d2(Vs.size());
    for (size_t k = 0; k < Vp.size(); ++k) {
      const int nn = (int)(k % ld) - pmb;
      const double sg = (nn & 1) ? -1.0 : 1.0;
      d1[k] = make_double2(Vp[k].x, -Vp[k].y);
      d2[k] = make_double2(Vs[k].x, -Vs[k].y);
      a1[k] = make_double2(sg * d1[k].x, sg * d1[k].y);
      a2[k] = make_double2(sg * d2[k].x, sg * d2[k].y);
    }
    if ((rc = upload(h, h->d_VpA_agg, a1.data(), a1.size()))) return rc;
    if ((rc = upload(h, h->d_VsA_agg, a2.data(), a2.size()))) return rc;
    if ((rc = upload(h, h->d_VpA_dis, d1.data(), d1.size()))) return rc;
    if ((rc = upload(h, h->d_VsA_dis, d2.data(), d2.size()))) return rc;
  }
  if (h->fmm_on) {
    ems::FmmPlan &F = h->fmm;
    std::vector<double2> pool(F.pool.size());
    for (size_t k = 0; k < pool.size(); ++k) pool[k] = make_double2(F.pool[k].real(), F.pool[k].imag());
    if ((rc = upload(h, h->d_pool, pool.data(), pool.size()))) return rc;
    if ((rc = upload(h, h->d_nbr_ptr, F.nbr_ptr.data(), F.nbr_ptr.size()))) return rc;
    if ((rc = upload(h, h->d_nbr_idx, F.nbr_idx.data(), std::max<size_t>(1, F.nbr_idx.size())))) return rc;
    {
      // partner offsets and orders per near pair: the near-field kernel reads
      // them by pair position, one dependent load fewer per partner
      std::vector<int64_t> noff(std::max<size_t>(1, F.nbr_idx.size()), 0);
      std::vector<int> npp(noff.size(), 0);
      for (size_t k = 0; k < F.nbr_idx.size(); ++k) {
        noff[k] = h->off[F.nbr_idx[k]];
        npp[k] = h->p[F.nbr_idx[k]];
      }
      if ((rc = upload(h, h->d_nbr_off, noff.data(), noff.size()))) return rc;
      if ((rc = upload(h, h->d_nbr_p, npp.data(), npp.size()))) return rc;
    }
    // near-pair symbols, tabulated once when they fit (forward near field)
    {
      const size_t nt = 4 * (size_t)ems::pm_bucket(h->pmax) + 1;
      const size_t bytes = (size_t)h->n_pairs * 2 * nt * sizeof(double2);
      size_t fre = 0, tot = 0;
      (void)hipMemGetInfo(&fre, &tot);
      if (h->n_pairs > 0 && bytes <= (size_t)16 << 30 && (double)bytes < 0.25 * (double)fre) {
        std::vector<int> tgt((size_t)h->n_pairs);
        for (int b = 0; b < h->n; ++b)
          for (int k = F.nbr_ptr[b]; k < F.nbr_ptr[b + 1]; ++k) tgt[k] = b;
        int *d_tgt = nullptr;
        if (hipMalloc(&h->d_nsym, bytes) == hipSuccess) {
          if ((rc = upload(h, d_tgt, tgt.data(), tgt.size()))) return rc;
          const hipError_t e = ems::launch_near_symbols(h, d_tgt, 0);
          const hipError_t e2 = hipDeviceSynchronize();
          dfree(d_tgt);
          HIPCHK(h, e);
          HIPCHK(h, e2);
        } else {
          (void)hipGetLastError();
          h->d_nsym = nullptr;
        }
      }
    }
    h->fmm_dev.assign(F.launches.size(), ems::FmmDev());
    {
      const ems::M2lPlan &Q = F.m2l;
      ems::M2lDev &D = h->m2l_dev;
      if ((rc = upload(h, D.g_P, Q.g_P.data(), Q.g_P.size()))) return rc;
      if ((rc = upload(h, D.g_G, Q.g_G.data(), Q.g_G.size()))) return rc;
      if ((rc = upload(h, D.g_nb, Q.g_nb.data(), Q.g_nb.size()))) return rc;
      if ((rc = upload(h, D.g_off, Q.g_off.data(), Q.g_off.size()))) return rc;
      if ((rc = upload(h, D.g_poff, Q.g_poff.data(), Q.g_poff.size()))) return rc;
      if ((rc = upload(h, D.tile_ptr, Q.tile_ptr.data(), Q.tile_ptr.size()))) return rc;
      if ((rc = upload(h, D.tile_box, Q.tile_box.data(), Q.tile_box.size()))) return rc;
      if ((rc = upload(h, D.ent_sym, Q.ent_sym.data(), Q.ent_sym.size()))) return rc;
      if ((rc = upload(h, D.ent_src, Q.ent_src.data(), Q.ent_src.size()))) return rc;
      if ((rc = upload(h, D.it_g, Q.it_g.data(), Q.it_g.size()))) return rc;
      if ((rc = upload(h, D.it_rt, Q.it_rt.data(), Q.it_rt.size()))) return rc;
      if ((rc = upload(h, D.it_tile, Q.it_tile.data(), Q.it_tile.size()))) return rc;
      if ((rc = upload(h, D.it_e0, Q.it_e0.data(), Q.it_e0.size()))) return rc;
      if ((rc = upload(h, D.it_e1, Q.it_e1.data(), Q.it_e1.size()))) return rc;
      if ((rc = upload(h, D.it_slot, Q.it_slot.data(), Q.it_slot.size()))) return rc;
    }
    static const char *names[] = {"fmm_p2m", "fmm_m2m", "fmm_l2p"};
    // M2L (matrix cores) and L2L launches named by tree level, top level 0
    static const char *m2l_names[] = {"fmm_m2l_0", "fmm_m2l_1", "fmm_m2l_2", "fmm_m2l_3",
                                      "fmm_m2l_4", "fmm_m2l_5", "fmm_m2l_6", "fmm_m2l_7",
                                      "fmm_m2l_8", "fmm_m2l_9", "fmm_m2l_10", "fmm_m2l_11",
                                      "fmm_m2l_12"};
    static const char *l2l_names[] = {"fmm_l2l_0", "fmm_l2l_1", "fmm_l2l_2", "fmm_l2l_3",
                                      "fmm_l2l_4", "fmm_l2l_5", "fmm_l2l_6", "fmm_l2l_7",
                                      "fmm_l2l_8", "fmm_l2l_9", "fmm_l2l_10", "fmm_l2l_11",
                                      "fmm_l2l_12"};
    int m2l_level = 0;
    for (size_t i = 0; i < F.launches.size(); ++i) {
      ems::FmmLaunch &L = F.launches[i];
      if (L.gemm_level >= 0) {
        m2l_level = L.gemm_level;
        L.name = m2l_names[std::min(m2l_level, 12)];
      } else if (L.in_kind == 0) L.name = names[0];
      else if (L.out_kind == 1) L.name = names[1];
      else if (L.out_kind == 2 && !L.accumulate) L.name = m2l_names[0];  // top level, tasks
      else if (L.out_kind == 2) L.name = l2l_names[std::min(m2l_level, 12)];
      else L.name = names[2];
      ems::FmmDev &D = h->fmm_dev[i];
      if ((rc = upload(h, D.ptr, L.ptr.data(), L.ptr.size()))) return rc;
      if ((rc = upload(h, D.in_P, L.in_P.data(), L.in_P.size()))) return rc;
      if ((rc = upload(h, D.sym_L, L.sym_L.data(), L.sym_L.size()))) return rc;
      if ((rc = upload(h, D.sgn, L.sgn.data(), L.sgn.size()))) return rc;
      if ((rc = upload(h, D.out_P, L.out_P.data(), L.out_P.size()))) return rc;
      if ((rc = upload(h, D.item_out, L.item_out.data(), L.item_out.size()))) return rc;
      if ((rc = upload(h, D.item_row0, L.item_row0.data(), L.item_row0.size()))) return rc;
      if ((rc = upload(h, D.item_t0, L.item_t0.data(), L.item_t0.size()))) return rc;
      if ((rc = upload(h, D.item_t1, L.item_t1.data(), L.item_t1.size()))) return rc;
      if ((rc = upload(h, D.item_slot, L.item_slot.data(), L.item_slot.size()))) return rc;
      if ((rc = upload(h, D.red_out, L.red_out.data(), L.red_out.size()))) return rc;
      if ((rc = upload(h, D.red_row0, L.red_row0.data(), L.red_row0.size()))) return rc;
      if ((rc = upload(h, D.red_slot0, L.red_slot0.data(), L.red_slot0.size()))) return rc;
      if ((rc = upload(h, D.red_g, L.red_g.data(), L.red_g.size()))) return rc;
      if ((rc = upload(h, D.in_base, L.in_base.data(), L.in_base.size()))) return rc;
      if ((rc = upload(h, D.sym_base, L.sym_base.data(), L.sym_base.size()))) return rc;
      if ((rc = upload(h, D.out_base, L.out_base.data(), L.out_base.size()))) return rc;
    }
  }
  // uniform truncation order: the kernels skip the per-mode range tests
  h->p_uniform = true;
  for (int i = 0; i < h->n; ++i)
    if (h->p[i] != h->pmax) h->p_uniform = false;
  // Depth order of the particles and the ranges of the truncated
  // contractions, the exponentials' node coefficients (register form), and,
  // unless switched off, the tabulated exponentials of each form that fits
  // the budget and free memory.  A form without tables forms its
  // exponentials in registers; without either, the vector-ALU kernels run.
  {
    ems::DepthCuts dc;
    h->depth_min = 1e300;
    for (int i = 0; i < h->n; ++i) h->depth_min = std::min(h->depth_min, -h->xy[2 * i + 1]);
    ems::depth_cuts(h->nodes, h->md, h->xy, h->pmax, h->somm.depth_cut, h->depth_min, dc);
    // coefficient-weighted kept fraction: the work of either contraction
    std::vector<double> pre(h->n + 1, 0.0);
    for (int i = 0; i < h->n; ++i) pre[i + 1] = pre[i] + 2.0 * h->p[dc.perm[i]] + 1.0;
    double kept = 0.0;
    for (size_t k = 0; k < dc.kcut.size(); ++k) kept += pre[dc.kcut[k]];
    h->depth_kept = kept / ((double)h->q * (double)h->ncoef);
    if ((rc = upload(h, h->d_sperm, dc.perm.data(), dc.perm.size()))) return rc;
    if ((rc = upload(h, h->d_kcut, dc.kcut.data(), dc.kcut.size()))) return rc;
    if ((rc = upload(h, h->d_jr, dc.jr.data(), dc.jr.size()))) return rc;
  }
  // the register form reduces the phase s_i y + xi_r x by Cody-Waite for
  // |phase| < 2^30 (|s| <= |xi| + k); clouds beyond it keep the tables
  double phase = 0.0;
  {
    double xm = 0.0, ym = 0.0, xim = 0.0;
    for (int i = 0; i < h->n; ++i) {
      xm = std::max(xm, std::fabs(h->xy[2 * i]));
      ym = std::max(ym, std::fabs(h->xy[2 * i + 1]));
    }
    for (const auto &z : h->nodes.xi) xim = std::max(xim, std::abs(z));
    phase = (xim + std::max(h->md.kp, h->md.ks)) * ym + xim * xm;
  }
  if (phase < 1.0e9) {
    HIPCHK(h, hipMalloc(&h->d_gco, sizeof(double4) * 8 * (size_t)h->q));
    HIPCHK(h, hipMalloc(&h->d_xys, sizeof(double2) * (size_t)h->n));
    HIPCHK(h, ems::launch_gen_coef(h, 0));
  }
  if (h->somm_tab) {
    const double gb = 4.0 * (double)h->q * (double)h->n * sizeof(double2) / 1e9;
    size_t fre = 0, tot = 0;
    (void)hipMemGetInfo(&fre, &tot);
    if (gb <= h->etab_budget_gb && gb * 1e9 < 0.6 * (double)fre && h->q <= 65535 &&
        h->n <= 65535) {
      const size_t half = (size_t)2 * h->q * h->n;
      if (hipMalloc(&h->d_Eagg, sizeof(double2) * half) != hipSuccess ||
          hipMalloc(&h->d_Edis, sizeof(double2) * half) != hipSuccess) {
        (void)hipGetLastError();
        dfree(h->d_Eagg);
        dfree(h->d_Edis);
      } else {
        // complex64 copies for the mixed form when they fit as well
        if (!h->somm_fp64 && 1.5 * gb <= h->etab_budget_gb && 1.5 * gb * 1e9 < 0.6 * (double)fre &&
            (hipMalloc(&h->d_Eagg32, sizeof(float2) * half) != hipSuccess ||
             hipMalloc(&h->d_Edis32, sizeof(float2) * half) != hipSuccess)) {
          (void)hipGetLastError();
          dfree(h->d_Eagg32);
          dfree(h->d_Edis32);
        }
        // conjugated tables of the adjoint when those fit too
        if (2.5 * gb <= h->etab_budget_gb && 2.5 * gb * 1e9 < 0.6 * (double)fre &&
            (hipMalloc(&h->d_EaggA, sizeof(double2) * half) != hipSuccess ||
             hipMalloc(&h->d_EdisA, sizeof(double2) * half) != hipSuccess)) {
          (void)hipGetLastError();
          dfree(h->d_EaggA);
          dfree(h->d_EdisA);
        }
        // table rows (aggregate) and columns (disaggregate) in depth order
        HIPCHK(h, ems::launch_etables(h, 0));
      }
    }
  }
  if ((rc = ensure_ws(h, 1))) return rc;
  HIPCHK(h, hipDeviceSynchronize());
  h->built = true;
  return EMS_OK;
}

int ems_get_info(const ems_handle *h, ems_build_info *out) {
  if (!h || !out) return EMS_ERR_ARG;
  out->n = h->n;
  out->p_max = h->pmax;
  out->n_coeff = h->ncoef;
  out->q = h->q;
  out->t_max = h->nodes.t_max;
  out->n_pairs = h->n_pairs;
  out->fmm_levels = h->fmm_on ? h->fmm.Lf - h->fmm.Lt + 1 : 0;
  out->fmm_m2l = h->fmm_on ? h->fmm.n_m2l : 0;
  out->kp = h->md.kp;
  out->ks = h->md.ks;
  out->kpb = h->md.kpb;
  out->ksb = h->md.ksb;
  out->somm_kept = ems::somm_mfma_ready(h, false) ? h->depth_kept : 1.0;
  out->mixed_near_fp64 = h->near_fp64 ? 1 : 0;
  out->mixed_somm_fp64 = (ems::somm_mfma_ready(h, false) && !ems::somm_mfma_fp32(h)) ? 1 : 0;
  return EMS_OK;
}

int ems_apply(ems_handle *h, const void *x, void *y, int32_t nrhs, int32_t flags,
              ems_stream_t stream) {
  if (!h || !x || !y || nrhs <= 0) return fail(h, EMS_ERR_ARG, "bad apply arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  if (x == y) return fail(h, EMS_ERR_ARG, "x and y must not alias");
  return apply_impl(h, (const double2 *)x, (double2 *)y, nrhs, flags, false,
                    (hipStream_t)stream);
}

int ems_apply_adjoint(ems_handle *h, const void *x, void *y, int32_t nrhs, int32_t flags,
                      ems_stream_t stream) {
  if (!h || !x || !y || nrhs <= 0) return fail(h, EMS_ERR_ARG, "bad apply arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  if (x == y) return fail(h, EMS_ERR_ARG, "x and y must not alias");
  return apply_impl(h, (const double2 *)x, (double2 *)y, nrhs, flags, true, (hipStream_t)stream);
}

int ems_incident(ems_handle *h, const ems_plane_wave *waves, int32_t nrhs, void *rhs,
                 ems_stream_t stream) {
  if (!h || !waves || !rhs || nrhs <= 0) return fail(h, EMS_ERR_ARG, "bad incident arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  hipStream_t st = (hipStream_t)stream;
  // host-side plane waves: {xi0, s_p, s_s, upgoing P, S, downgoing P, S}
  std::vector<double2> pw(7 * (size_t)nrhs);
  for (int r = 0; r < nrhs; ++r) {
    PwParts pp;
    const int rc = plane_wave_parts(h->md, waves[r], pp, h->err);
    if (rc) return rc;
    cd up[2] = {0.0, 0.0}, dn[2] = {0.0, 0.0};
    for (const PwComp &c : pp.comp) {
      if (c.layer != 0) continue;
      if (c.up) up[c.kind] += c.A;
      else dn[c.kind] += c.A;
    }
    const cd v[7] = {cd(pp.xi0, 0.0), pp.s4[0], pp.s4[1], up[0], up[1], dn[0], dn[1]};
    for (int k2 = 0; k2 < 7; ++k2) pw[7 * (size_t)r + k2] = make_double2(v[k2].real(), v[k2].imag());
  }
  const size_t nvec = (size_t)nrhs * h->ncoef;
  int rc = ensure_tmp(h, sizeof(double2) * nvec + sizeof(double2) * pw.size());
  if (rc) return rc;
  double2 *c = h->d_tmp;
  double2 *dpw = h->d_tmp + nvec;
  HIPCHK(h, hipMemcpyAsync(dpw, pw.data(), pw.size() * sizeof(double2), hipMemcpyHostToDevice, st));
  HIPCHK(h, ems::launch_incident_pw(h, dpw, nrhs, c, st));
  HIPCHK(h, ems::launch_s_apply(h, c, (double2 *)rhs, nrhs, false, st));
  HIPCHK(h, hipStreamSynchronize(st));
  return EMS_OK;
}

int ems_eval_background(ems_handle *h, const ems_plane_wave *waves, int32_t nrhs, int32_t npts,
                        const double *pts, void *u, ems_stream_t stream) {
  if (!h || !waves || !pts || !u || nrhs <= 0 || npts <= 0)
    return fail(h, EMS_ERR_ARG, "bad background arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  hipStream_t st = (hipStream_t)stream;
  {
    std::vector<double> hp(2 * (size_t)npts);
    HIPCHK(h, hipMemcpyAsync(hp.data(), pts, sizeof(double) * hp.size(), hipMemcpyDeviceToHost,
                             st));
    HIPCHK(h, hipStreamSynchronize(st));
    for (int i = 0; i < npts; ++i) {
      if (!std::isfinite(hp[2 * i]) || !std::isfinite(hp[2 * i + 1]))
        return fail(h, EMS_ERR_NUMERIC, "non-finite point");
      if (hp[2 * i + 1] == 0.0) return fail(h, EMS_ERR_GEOMETRY, "point on the interface (y = 0)");
    }
  }
  std::vector<double2> comp(18 * (size_t)nrhs);
  for (int r = 0; r < nrhs; ++r) {
    PwParts pp;
    const int rc = plane_wave_parts(h->md, waves[r], pp, h->err);
    if (rc) return rc;
    for (int c = 0; c < 6; ++c) {
      double2 *C = comp.data() + ((size_t)r * 6 + c) * 3;
      if (c < (int)pp.comp.size()) {
        const PwComp &k = pp.comp[c];
        C[0] = make_double2(k.A.real(), k.A.imag());
        C[1] = make_double2(k.q.real(), k.q.imag());
        C[2] = make_double2(pp.xi0, 2.0 * k.layer + k.kind);
      } else {
        C[0] = C[1] = make_double2(0.0, 0.0);
        C[2] = make_double2(0.0, -1.0);
      }
    }
  }
  int rc = ensure_tmp(h, sizeof(double2) * comp.size());
  if (rc) return rc;
  HIPCHK(h, hipMemcpyAsync(h->d_tmp, comp.data(), comp.size() * sizeof(double2),
                           hipMemcpyHostToDevice, st));
  HIPCHK(h, ems::launch_background(nrhs, npts, pts, h->d_tmp, (double2 *)u, st));
  HIPCHK(h, hipStreamSynchronize(st));
  return EMS_OK;
}

int ems_incident_point(ems_handle *h, const ems_point_source *src, int32_t nrhs, void *rhs,
                       ems_stream_t stream) {
  if (!h || !src || !rhs || nrhs <= 0) return fail(h, EMS_ERR_ARG, "bad point-source arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  hipStream_t st = (hipStream_t)stream;
  double xlo = HUGE_VAL, xhi = -HUGE_VAL, dlo = HUGE_VAL, dhi = -HUGE_VAL;
  for (int m = 0; m < h->n; ++m) {
    xlo = std::min(xlo, h->xy[2 * m]);
    xhi = std::max(xhi, h->xy[2 * m]);
    dlo = std::min(dlo, -h->xy[2 * m + 1]);
    dhi = std::max(dhi, -h->xy[2 * m + 1]);
  }
  PointNodes pn;
  int rc = point_nodes(h, src, nrhs, xlo, xhi, dlo, dhi, pn);
  if (rc) return rc;
  const int q = (int)pn.nt.xi.size();
  const size_t nvec = (size_t)nrhs * h->ncoef;
  const size_t nd3 = 3 * (size_t)q, na = 2 * (size_t)q * nrhs;
  const size_t nv = 2 * (size_t)q * (2 * h->pmax + 1);
  if ((rc = ensure_tmp(h, sizeof(double2) * (nvec + nd3 + na + nv)))) return rc;
  std::vector<double2> nd(nd3), amp(na);
  for (int jj = 0; jj < q; ++jj)
    for (int k = 0; k < 3; ++k) nd[3 * (size_t)jj + k] = pn.nd[5 * (size_t)jj + k];
  for (int r = 0; r < nrhs; ++r)
    for (int jj = 0; jj < q; ++jj)
      for (int k = 0; k < 2; ++k)
        amp[((size_t)r * q + jj) * 2 + k] = pn.amp[((size_t)r * q + jj) * 4 + k];
  double2 *c = h->d_tmp, *dnd = c + nvec, *damp = dnd + nd3;
  HIPCHK(h, hipMemcpyAsync(dnd, nd.data(), nd3 * sizeof(double2), hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(damp, amp.data(), na * sizeof(double2), hipMemcpyHostToDevice, st));
  {
    ems::ProfScope ps(h, "point_local", st);
    HIPCHK(h, ems::launch_point_local(h, q, dnd, damp, nrhs, c, damp + na, st));
  }
  HIPCHK(h, ems::launch_s_apply(h, c, (double2 *)rhs, nrhs, false, st));
  HIPCHK(h, hipStreamSynchronize(st));
  return EMS_OK;
}

int ems_eval_background_point(ems_handle *h, const ems_point_source *src, int32_t nrhs,
                              int32_t npts, const double *pts, void *u, ems_stream_t stream) {
  if (!h || !src || !pts || !u || nrhs <= 0 || npts <= 0)
    return fail(h, EMS_ERR_ARG, "bad point-source field arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> hp(2 * (size_t)npts);
  HIPCHK(h, hipMemcpyAsync(hp.data(), pts, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  double xlo = HUGE_VAL, xhi = -HUGE_VAL, dlo = HUGE_VAL, dhi = -HUGE_VAL;
  for (int i = 0; i < npts; ++i) {
    const double x = hp[2 * i], y = hp[2 * i + 1];
    if (!std::isfinite(x) || !std::isfinite(y)) return fail(h, EMS_ERR_NUMERIC, "non-finite point");
    if (y == 0.0) return fail(h, EMS_ERR_GEOMETRY, "point on the interface (y = 0)");
    for (int r = 0; r < nrhs; ++r)
      if (std::hypot(x - src[r].x0, y - src[r].y0) < 1e-9)
        return fail(h, EMS_ERR_GEOMETRY, "point at a source");
    xlo = std::min(xlo, x);
    xhi = std::max(xhi, x);
    dlo = std::min(dlo, std::fabs(y));
    dhi = std::max(dhi, std::fabs(y));
  }
  PointNodes pn;
  int rc = point_nodes(h, src, nrhs, xlo, xhi, dlo, dhi, pn);
  if (rc) return rc;
  const int q = (int)pn.nt.xi.size();
  const size_t nd5 = pn.nd.size(), na = pn.amp.size(), ns = 2 * (size_t)nrhs;
  if ((rc = ensure_tmp(h, sizeof(double2) * (nd5 + na + ns)))) return rc;
  std::vector<double> sv(4 * (size_t)nrhs);
  for (int r = 0; r < nrhs; ++r) {
    sv[4 * r] = src[r].x0;
    sv[4 * r + 1] = src[r].y0;
    sv[4 * r + 2] = src[r].alpha1;
    sv[4 * r + 3] = src[r].alpha2;
  }
  double2 *dnd = h->d_tmp, *damp = dnd + nd5;
  double *dsrc = reinterpret_cast<double *>(damp + na);
  HIPCHK(h, hipMemcpyAsync(dnd, pn.nd.data(), nd5 * sizeof(double2), hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(damp, pn.amp.data(), na * sizeof(double2), hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(dsrc, sv.data(), sv.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(h, ems::launch_point_field(h, q, dnd, damp, dsrc, nrhs, npts, pts, (double2 *)u, st));
  HIPCHK(h, hipStreamSynchronize(st));
  return EMS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// GMRES
namespace {

struct Givens {
  std::vector<cd> cs, sn, g;
  std::vector<std::vector<cd>> H;  // columns
};

// Restarted GMRES on nrhs systems in lock-step.  op(x, y) applies the
// operator A to nrhs vectors; with prec (use_prec) the Krylov space is built
// on A M^{-1} (right preconditioning: the residual stays that of A) and the
// update is x += M^{-1} V y.  Every sweep starts from the true residual
// b - A x, so the stopping test is always on a computed residual.  x is
// updated in place (initial guess taken as given; x_zero skips the first
// product).  The estimated relative residual of every iteration (largest over
// the systems, times hist_scale) is appended to h->hist.
// stall > 0 (inner solves of the mixed refinement, whose FP32 products put a
// floor under the reachable residual): a sweep also ends when its estimate
// fell by less than 10 % over the last `stall` iterations.
template <typename TB, typename Op, typename Prec>
int gmres_basis(ems_handle *h, Op op, Prec prec, bool use_prec, const double2 *b, double2 *x,
                int nrhs, double tol, int restart, int maxit, bool x_zero, hipStream_t st,
                int &iters, double &relres, std::vector<double> &bnorm_out, double hist_scale,
                int stall) {
  const int64_t n = h->ncoef;
  const size_t vec = (size_t)n;
  restart = std::max(1, std::min(restart, maxit));
  // basis V[k][r][n] (complex64 in the inner solves of the mixed refinement)
  const size_t vbytes = sizeof(TB) * (size_t)(restart + 1) * nrhs * vec;
  if (h->V_bytes < vbytes) {
    if (h->d_V) (void)hipFree(h->d_V);
    h->d_V = nullptr;
    h->V_bytes = 0;
    HIPCHK(h, hipMalloc(&h->d_V, vbytes));
    h->V_bytes = vbytes;
  }
  constexpr bool F32 = std::is_same<TB, float2>::value;
  int rc = ensure_tmp(h, sizeof(double2) * (F32 ? 3 : 2) * nrhs * vec);
  if (rc) return rc;
  if (use_prec && (rc = ensure_pcz(h, nrhs))) return rc;
  // d_h, d_h2 [restart + 2] each, the norm result (restart + 2 + 8 slots
  // before the partials), then up to restart + 1 reduced vectors of
  // kRedBlocks complex partials each
  rc = ensure_red(h, sizeof(double2) * (3 * (size_t)(restart + 2) + 8 +
                                        (size_t)(restart + 1) * ems::kRedBlocks));
  if (rc) return rc;
  double2 *W = h->d_tmp;                 // [nrhs][n] operator output
  double2 *Z = h->d_pcz, *Z2 = h->d_pcz ? h->d_pcz + (size_t)nrhs * vec : nullptr;
  double2 *d_h = reinterpret_cast<double2 *>(h->d_red);  // device coefficients
  double2 *d_h2 = d_h + (restart + 2);
  double *d_nrm = reinterpret_cast<double *>(d_h2 + (restart + 2));
  double *scratch = reinterpret_cast<double *>(d_h2 + 2 * (restart + 2) + 8);
  TB *Vb = reinterpret_cast<TB *>(h->d_V);
  auto Vk = [&](int k, int r) { return Vb + ((size_t)k * nrhs + r) * vec; };
  // the operator's input: the basis vectors themselves, or widened to FP64
  double2 *Vin = h->d_tmp + (size_t)2 * nrhs * vec;
  auto opnd = [&](int k) -> const double2 * {
    if constexpr (F32) {
      (void)ems::launch_widen(Vk(k, 0), Vin, (int64_t)nrhs * n, st);
      return Vin;
    } else {
      return Vk(k, 0);
    }
  };
  const int64_t ldv = (int64_t)nrhs * n;

  std::vector<double> bnorm(nrhs), beta(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    HIPCHK(h, ems::launch_norm2(b + r * vec, n, d_nrm, scratch, st));
    HIPCHK(h, hipMemcpyAsync(&bnorm[r], d_nrm, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
  }
  bnorm_out = bnorm;
  std::vector<double> rel(nrhs, 0.0);
  iters = 0;
  relres = 0.0;
  bool first = true;
  while (true) {
    // true residual W = b - A x (x = 0 on the first sweep when x_zero)
    if (first && x_zero) {
      for (int r = 0; r < nrhs; ++r)
        HIPCHK(h, hipMemcpyAsync(W + r * vec, b + r * vec, sizeof(double2) * vec,
                                 hipMemcpyDeviceToDevice, st));
    } else {
      rc = op(x, W);
      if (rc) return rc;
      for (int r = 0; r < nrhs; ++r) {
        HIPCHK(h, ems::launch_scale(W + r * vec, n, -1.0, st));
        HIPCHK(h, ems::launch_axpy(W + r * vec, b + r * vec, n, 1.0, st));
      }
    }
    first = false;
    std::vector<Givens> G(nrhs);
    std::vector<int> kk(nrhs, 0);
    std::vector<bool> active(nrhs, false);
    bool any = false;
    relres = 0.0;
    for (int r = 0; r < nrhs; ++r) {
      HIPCHK(h, ems::launch_norm2(W + r * vec, n, d_nrm, scratch, st));
      HIPCHK(h, hipMemcpyAsync(&beta[r], d_nrm, sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(h, hipStreamSynchronize(st));
      rel[r] = bnorm[r] > 0 ? beta[r] / bnorm[r] : 0.0;
      relres = std::max(relres, rel[r]);
      if (bnorm[r] == 0.0 || rel[r] <= tol) continue;
      active[r] = true;
      any = true;
    }
    if (!any || iters >= maxit) break;
    for (int r = 0; r < nrhs; ++r) {
      if (!active[r]) continue;
      G[r].g.assign(restart + 1, cd(0.0));
      G[r].g[0] = beta[r];
      G[r].cs.assign(restart, 0.0);
      G[r].sn.assign(restart, 0.0);
      G[r].H.assign(restart, std::vector<cd>(restart + 1, 0.0));
      HIPCHK(h, ems::launch_copy_scaled(W + r * vec, Vk(0, r), n, 1.0 / beta[r], st));
    }
    int k = 0;
    std::vector<double> sweep_hist;
    bool stalled = false;
    for (; k < restart && iters < maxit; ++k) {
      // W = A V_k, or A M^{-1} V_k (all right-hand sides; inactive ones are ignored)
      const double2 *vin = opnd(k);
      HIPCHK(h, hipGetLastError());
      if (use_prec) {
        rc = prec(vin, Z);
        if (rc) return rc;
        rc = op(Z, W);
      } else {
        rc = op(vin, W);
      }
      if (rc) return rc;
      ++iters;
      bool all_done = true;
      for (int r = 0; r < nrhs; ++r) {
        if (!active[r]) continue;
        double2 *w = W + r * vec;
        // classical Gram-Schmidt, repeated once when the first pass cancels
        // more than 30 % of ||w|| ("twice is enough": a second pass then
        // restores orthogonality to working precision)
        double nrm0 = 0, nrm = 0;
        HIPCHK(h, ems::launch_norm2(w, n, d_nrm + 1, scratch, st));
        HIPCHK(h, ems::launch_mdot(Vk(0, r), ldv, k + 1, w, n, d_h, scratch, st));
        HIPCHK(h, ems::launch_mupdate(Vk(0, r), ldv, k + 1, d_h, w, n, st));
        HIPCHK(h, ems::launch_norm2(w, n, d_nrm, scratch, st));
        std::vector<double2> h1(k + 1), h2(k + 1, make_double2(0.0, 0.0));
        HIPCHK(h, hipMemcpyAsync(h1.data(), d_h, sizeof(double2) * (k + 1), hipMemcpyDeviceToHost, st));
        HIPCHK(h, hipMemcpyAsync(&nrm, d_nrm, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(h, hipMemcpyAsync(&nrm0, d_nrm + 1, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(h, hipStreamSynchronize(st));
        if (!(nrm > 0.7 * nrm0)) {
          ++h->reorth;
          HIPCHK(h, ems::launch_mdot(Vk(0, r), ldv, k + 1, w, n, d_h2, scratch, st));
          HIPCHK(h, ems::launch_mupdate(Vk(0, r), ldv, k + 1, d_h2, w, n, st));
          HIPCHK(h, ems::launch_norm2(w, n, d_nrm, scratch, st));
          HIPCHK(h, hipMemcpyAsync(h2.data(), d_h2, sizeof(double2) * (k + 1), hipMemcpyDeviceToHost, st));
          HIPCHK(h, hipMemcpyAsync(&nrm, d_nrm, sizeof(double), hipMemcpyDeviceToHost, st));
          HIPCHK(h, hipStreamSynchronize(st));
        }
        std::vector<cd> col(k + 2);
        for (int i = 0; i <= k; ++i) col[i] = cd(h1[i].x + h2[i].x, h1[i].y + h2[i].y);
        col[k + 1] = nrm;
        if (nrm > 0) HIPCHK(h, ems::launch_copy_scaled(w, Vk(k + 1, r), n, 1.0 / nrm, st));
        Givens &g = G[r];
        for (int i = 0; i < k; ++i) {
          const cd t = g.cs[i] * col[i] + g.sn[i] * col[i + 1];
          col[i + 1] = -std::conj(g.sn[i]) * col[i] + std::conj(g.cs[i]) * col[i + 1];
          col[i] = t;
        }
        const double den = std::hypot(std::abs(col[k]), std::abs(col[k + 1]));
        if (den == 0) {
          g.cs[k] = 1.0;
          g.sn[k] = 0.0;
        } else {
          g.cs[k] = std::conj(col[k]) / den;
          g.sn[k] = std::conj(col[k + 1]) / den;
        }
        col[k] = g.cs[k] * col[k] + g.sn[k] * col[k + 1];
        col[k + 1] = 0.0;
        g.g[k + 1] = -std::conj(g.sn[k]) * g.g[k];
        g.g[k] = g.cs[k] * g.g[k];
        g.H[k] = col;
        kk[r] = k + 1;
        rel[r] = std::abs(g.g[k + 1]) / bnorm[r];
        if (rel[r] <= tol || nrm == 0) active[r] = false;
        else all_done = false;
      }
      double hmax = 0.0;
      for (int r = 0; r < nrhs; ++r) hmax = std::max(hmax, rel[r]);
      h->hist.push_back(hmax * hist_scale);
      if (h->progress && h->progress_every > 0 && (int)h->hist.size() % h->progress_every == 0)
        h->progress((int32_t)h->hist.size(), hmax * hist_scale, h->progress_user);
      sweep_hist.push_back(hmax);
      if (stall > 0 && (int)sweep_hist.size() > stall &&
          hmax > 0.9 * sweep_hist[sweep_hist.size() - 1 - stall])
        stalled = true;
      if (all_done || stalled) {
        ++k;
        break;
      }
    }
    // x += V y (or M^{-1} V y) for every system that took steps in this sweep
    if (use_prec) HIPCHK(h, hipMemsetAsync(Z, 0, sizeof(double2) * vec * nrhs, st));
    for (int r = 0; r < nrhs; ++r) {
      const int kr = kk[r];
      if (kr == 0) continue;
      std::vector<cd> y(kr);
      Givens &g = G[r];
      for (int i = kr - 1; i >= 0; --i) {
        cd s = g.g[i];
        for (int j = i + 1; j < kr; ++j) s -= g.H[j][i] * y[j];
        y[i] = s / g.H[i][i];
      }
      std::vector<double2> yd(kr);
      for (int i = 0; i < kr; ++i) yd[i] = make_double2(y[i].real(), y[i].imag());
      HIPCHK(h, hipMemcpyAsync(d_h, yd.data(), sizeof(double2) * kr, hipMemcpyHostToDevice, st));
      HIPCHK(h, ems::launch_maccum(Vk(0, r), ldv, kr, d_h, use_prec ? Z + r * vec : x + r * vec,
                                   n, st));
      HIPCHK(h, hipStreamSynchronize(st));
    }
    if (use_prec) {
      rc = prec(Z, Z2);
      if (rc) return rc;
      for (int r = 0; r < nrhs; ++r)
        if (kk[r] > 0) HIPCHK(h, ems::launch_axpy(x + r * vec, Z2 + r * vec, n, 1.0, st));
    }
    if (stalled) {
      // report the residual of the stalled sweep's iterate
      rc = op(x, W);
      if (rc) return rc;
      relres = 0.0;
      for (int r = 0; r < nrhs; ++r) {
        HIPCHK(h, ems::launch_scale(W + r * vec, n, -1.0, st));
        HIPCHK(h, ems::launch_axpy(W + r * vec, b + r * vec, n, 1.0, st));
        double nr = 0.0;
        HIPCHK(h, ems::launch_norm2(W + r * vec, n, d_nrm, scratch, st));
        HIPCHK(h, hipMemcpyAsync(&nr, d_nrm, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(h, hipStreamSynchronize(st));
        if (bnorm[r] > 0) relres = std::max(relres, nr / bnorm[r]);
      }
      break;
    }
  }
  return EMS_OK;
}

// GMRES with an FP64 basis, or (f32_basis) a complex64 one: half the
// Gram-Schmidt traffic, for the inner solves of the mixed refinement whose
// tolerance stays far above the FP32 orthogonality level.
template <typename Op, typename Prec>
int gmres_run(ems_handle *h, Op op, Prec prec, bool use_prec, const double2 *b, double2 *x,
              int nrhs, double tol, int restart, int maxit, bool x_zero, hipStream_t st,
              int &iters, double &relres, std::vector<double> &bnorm_out, double hist_scale,
              int stall = 0, bool f32_basis = false) {
  if (f32_basis)
    return gmres_basis<float2>(h, op, prec, use_prec, b, x, nrhs, tol, restart, maxit, x_zero, st,
                               iters, relres, bnorm_out, hist_scale, stall);
  return gmres_basis<double2>(h, op, prec, use_prec, b, x, nrhs, tol, restart, maxit, x_zero, st,
                              iters, relres, bnorm_out, hist_scale, stall);
}

// Cholesky G = R^H R of an s x s Hermitian matrix (row-major), R upper; false
// when a pivot falls below rel_piv times the largest diagonal entry (the
// block is numerically rank deficient).
bool chol_upper(const std::vector<cd> &G, int s, std::vector<cd> &R, double rel_piv) {
  R.assign((size_t)s * s, cd(0.0));
  double gmax = 0.0;
  for (int i = 0; i < s; ++i) gmax = std::max(gmax, G[(size_t)i * s + i].real());
  for (int i = 0; i < s; ++i) {
    double d = G[(size_t)i * s + i].real();
    for (int l = 0; l < i; ++l) d -= std::norm(R[(size_t)l * s + i]);
    if (!(d > rel_piv * gmax) || !std::isfinite(d)) return false;
    const double rii = std::sqrt(d);
    R[(size_t)i * s + i] = rii;
    for (int c = i + 1; c < s; ++c) {
      cd v = G[(size_t)i * s + c];
      for (int l = 0; l < i; ++l) v -= std::conj(R[(size_t)l * s + i]) * R[(size_t)l * s + c];
      R[(size_t)i * s + c] = v / rii;
    }
  }
  return true;
}

// Inverse of an upper triangular s x s matrix (row-major).
std::vector<cd> inv_upper(const std::vector<cd> &R, int s) {
  std::vector<cd> X((size_t)s * s, cd(0.0));
  for (int c = 0; c < s; ++c) {
    X[(size_t)c * s + c] = 1.0 / R[(size_t)c * s + c];
    for (int i = c - 1; i >= 0; --i) {
      cd v = 0.0;
      for (int l = i + 1; l <= c; ++l) v += R[(size_t)i * s + l] * X[(size_t)l * s + c];
      X[(size_t)i * s + c] = -v / R[(size_t)i * s + i];
    }
  }
  return X;
}

std::vector<double2> to_dev_layout(const std::vector<cd> &a) {
  std::vector<double2> o(a.size());
  for (size_t i = 0; i < a.size(); ++i) o[i] = make_double2(a[i].real(), a[i].imag());
  return o;
}

// Block GMRES (Section 4.2 and 5.2 systems, several right-hand sides sharing
// one Krylov space): for the s <= 64 columns of b, the block Arnoldi process
// on A M^{-1} (right preconditioning, or A) with block classical
// Gram-Schmidt run twice (bdot / baxpy on the matrix cores) and the new block
// orthonormalised by Cholesky QR run twice; the block upper Hessenberg matrix
// is reduced by Givens rotations on the host (its s sub-diagonals), so every
// column's residual estimate is known after each block step.  A cycle ends
// after mblk block steps, when every column meets tol, or at a breakdown;
// x += M^{-1} V Y, then the next cycle starts from the true residual of the
// columns that still miss tol (converged columns leave the block).
// op(in, out, cnt) / prec(in, out, cnt) act on cnt stacked vectors.
template <typename Op, typename Prec>
int block_gmres_run(ems_handle *h, Op op, Prec prec, bool use_prec, const double2 *b, double2 *x,
                    int s0, double tol, int mblk, int maxit, hipStream_t st, int &iters,
                    double &relres) {
  const int64_t n = h->ncoef;
  const size_t vec = (size_t)n;
  mblk = std::max(1, std::min(mblk, maxit));
  const size_t vbytes = sizeof(double2) * (size_t)(mblk + 1) * s0 * vec;
  if (h->V_bytes < vbytes) {
    if (h->d_V) (void)hipFree(h->d_V);
    h->d_V = nullptr;
    h->V_bytes = 0;
    HIPCHK(h, hipMalloc(&h->d_V, vbytes));
    h->V_bytes = vbytes;
  }
  int rc = ensure_tmp(h, sizeof(double2) * 2 * s0 * vec);
  if (rc) return rc;
  if (use_prec && (rc = ensure_pcz(h, s0))) return rc;
  const int kmax = (mblk + 1) * s0;
  const size_t hlen = (size_t)kmax * s0;
  const size_t plen = (size_t)ems::bdot_chunks(kmax, n) * kmax * s0 + (size_t)32768 * s0;
  rc = ensure_red(h, sizeof(double2) * (hlen + plen + s0 * s0) + 8 * sizeof(double) +
                         sizeof(double2) * ems::kRedBlocks);
  if (rc) return rc;
  double2 *Hd = reinterpret_cast<double2 *>(h->d_red);
  double2 *part = Hd + hlen;
  double2 *Sd = part + plen;  // s x s factors on device
  double *d_nrm = reinterpret_cast<double *>(Sd + (size_t)s0 * s0);
  double *scratch = d_nrm + 8;
  double2 *W = h->d_tmp, *Qv = h->d_tmp + (size_t)s0 * vec;
  double2 *Z = h->d_pcz;
  double2 *V = h->d_V;

  auto col_norms = [&](const double2 *v, int cnt, std::vector<double> &out) -> int {
    out.assign(cnt, 0.0);
    for (int c = 0; c < cnt; ++c) {
      HIPCHK(h, ems::launch_norm2(v + (size_t)c * vec, n, d_nrm, scratch, st));
      HIPCHK(h, hipMemcpyAsync(&out[c], d_nrm, sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(h, hipStreamSynchronize(st));
    }
    return EMS_OK;
  };
  auto gram = [&](const double2 *A, int k, const double2 *B, int cnt, std::vector<cd> &out) -> int {
    HIPCHK(h, ems::launch_bdot(A, k, B, cnt, n, Hd, part, st));
    std::vector<double2> t((size_t)k * cnt);
    HIPCHK(h, hipMemcpyAsync(t.data(), Hd, sizeof(double2) * t.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    out.resize(t.size());
    for (size_t i = 0; i < t.size(); ++i) out[i] = cd(t[i].x, t[i].y);
    return EMS_OK;
  };
  // out = in * F (cnt vectors, F cnt x cnt row-major on the host)
  auto transform = [&](const double2 *in, int cnt, const std::vector<cd> &F, double2 *out) -> int {
    const auto f = to_dev_layout(F);
    HIPCHK(h, hipMemcpyAsync(Sd, f.data(), sizeof(double2) * f.size(), hipMemcpyHostToDevice, st));
    HIPCHK(h, ems::launch_baxpy(in, cnt, Sd, cnt, n, out, 1.0, 0.0, st));
    return EMS_OK;
  };
  // Cholesky QR twice, the first on the column-scaled Gram matrix: out =
  // in T^{-1} orthonormal, T upper (in is used as scratch); ok = false when a
  // scaled pivot falls below 1e-14 (the block is numerically rank deficient)
  auto cholqr2 = [&](double2 *in, int cnt, double2 *out, std::vector<cd> &T, bool &ok) -> int {
    std::vector<cd> G, R1, R2;
    ok = false;
    int r;
    if ((r = gram(in, cnt, in, cnt, G))) return r;
    std::vector<double> d(cnt);
    for (int i = 0; i < cnt; ++i) {
      d[i] = std::sqrt(std::max(G[(size_t)i * cnt + i].real(), 0.0));
      if (!(d[i] > 0)) return EMS_OK;
    }
    for (int i = 0; i < cnt; ++i)
      for (int c = 0; c < cnt; ++c) G[(size_t)i * cnt + c] /= d[i] * d[c];
    if (!chol_upper(G, cnt, R1, 1e-14)) return EMS_OK;
    std::vector<cd> F = inv_upper(R1, cnt);
    for (int i = 0; i < cnt; ++i)
      for (int c = 0; c < cnt; ++c) F[(size_t)i * cnt + c] /= d[i];
    if ((r = transform(in, cnt, F, out))) return r;
    for (int i = 0; i < cnt; ++i)
      for (int c = 0; c < cnt; ++c) R1[(size_t)i * cnt + c] *= d[c];
    if ((r = gram(out, cnt, out, cnt, G))) return r;
    if (!chol_upper(G, cnt, R2, 1e-14)) return EMS_OK;
    if ((r = transform(out, cnt, inv_upper(R2, cnt), in))) return r;
    HIPCHK(h, hipMemcpyAsync(out, in, sizeof(double2) * cnt * vec, hipMemcpyDeviceToDevice, st));
    T.assign((size_t)cnt * cnt, cd(0.0));
    for (int i = 0; i < cnt; ++i)
      for (int c = i; c < cnt; ++c) {
        cd v = 0.0;
        for (int l = i; l <= c; ++l) v += R2[(size_t)i * cnt + l] * R1[(size_t)l * cnt + c];
        T[(size_t)i * cnt + c] = v;
      }
    ok = true;
    return EMS_OK;
  };

  std::vector<double> bnorm;
  if ((rc = col_norms(b, s0, bnorm))) return rc;
  iters = 0;
  relres = 0.0;
  bool first = true;
  while (true) {
    // true residual of every column, the active ones gathered into W
    std::vector<double> rn;
    if (first) {
      HIPCHK(h, hipMemcpyAsync(Qv, b, sizeof(double2) * s0 * vec, hipMemcpyDeviceToDevice, st));
    } else {
      if ((rc = op(x, Qv, s0))) return rc;
      for (int c = 0; c < s0; ++c) {
        HIPCHK(h, ems::launch_scale(Qv + c * vec, n, -1.0, st));
        HIPCHK(h, ems::launch_axpy(Qv + c * vec, b + c * vec, n, 1.0, st));
      }
    }
    first = false;
    if ((rc = col_norms(Qv, s0, rn))) return rc;
    std::vector<int> act;
    relres = 0.0;
    for (int c = 0; c < s0; ++c) {
      const double rel = bnorm[c] > 0 ? rn[c] / bnorm[c] : 0.0;
      relres = std::max(relres, rel);
      if (bnorm[c] > 0 && rel > tol) act.push_back(c);
    }
    if (act.empty() || iters >= maxit) break;
    // The cycle's block: residual columns taken by decreasing relative size
    // while they stay independent (pivoted Cholesky of the column-scaled Gram
    // matrix, scaled pivot above 1e-10); a column close to the span of the
    // others waits for a later cycle.
    {
      std::sort(act.begin(), act.end(), [&](int a, int c) {
        return rn[a] / bnorm[a] > rn[c] / bnorm[c];
      });
      const int na = (int)act.size();
      for (int a = 0; a < na; ++a)
        HIPCHK(h, hipMemcpyAsync(W + (size_t)a * vec, Qv + (size_t)act[a] * vec,
                                 sizeof(double2) * vec, hipMemcpyDeviceToDevice, st));
      std::vector<cd> G;
      if ((rc = gram(W, na, W, na, G))) return rc;
      std::vector<double> d(na);
      for (int a = 0; a < na; ++a) d[a] = std::sqrt(std::max(G[(size_t)a * na + a].real(), 1e-300));
      std::vector<int> keep;          // positions in act
      std::vector<std::vector<cd>> L;  // rows of the partial factor (scaled)
      for (int a = 0; a < na; ++a) {
        std::vector<cd> row(keep.size());
        // row a of the lower factor of the scaled Gram matrix over the kept columns
        for (size_t t = 0; t < keep.size(); ++t) {
          cd v = G[(size_t)a * na + keep[t]] / (d[a] * d[keep[t]]);
          for (size_t l = 0; l < t; ++l) v -= row[l] * std::conj(L[t][l]);
          row[t] = v / L[t][t];
        }
        double piv = 1.0;
        for (const auto &v : row) piv -= std::norm(v);
        if (piv > 1e-10) {
          row.push_back(std::sqrt(piv));
          L.push_back(row);
          keep.push_back(a);
        }
      }
      std::vector<int> sel;
      for (int a : keep) sel.push_back(act[a]);
      act.swap(sel);
    }
    const int sa = (int)act.size();
    for (int a = 0; a < sa; ++a)
      HIPCHK(h, hipMemcpyAsync(W + (size_t)a * vec, Qv + (size_t)act[a] * vec,
                               sizeof(double2) * vec, hipMemcpyDeviceToDevice, st));
    // W = V_0 beta
    std::vector<cd> beta;
    bool ok = false;
    if ((rc = cholqr2(W, sa, V, beta, ok))) return rc;
    if (!ok) return fail(h, EMS_ERR_NUMERIC, "block GMRES: residual block is rank deficient");
    // band Hessenberg columns, their rotations, and the rotated right-hand sides
    const int ncol = mblk * sa;
    std::vector<std::vector<cd>> Hc;
    std::vector<cd> rcs((size_t)ncol * sa), rsn((size_t)ncol * sa);
    std::vector<cd> Gr((size_t)(mblk + 1) * sa * sa, cd(0.0));  // [row][column]
    for (int i = 0; i < sa; ++i)
      for (int c = 0; c < sa; ++c) Gr[(size_t)i * sa + c] = beta[(size_t)i * sa + c];
    auto rotate = [&](cd cs, cd sn, cd &u, cd &v) {
      const cd t = cs * u + sn * v;
      v = -std::conj(sn) * u + std::conj(cs) * v;
      u = t;
    };
    int J = 0;  // completed block steps of this cycle
    bool breakdown = false;
    for (int j = 0; j < mblk && iters < maxit; ++j) {
      const double2 *Vj = V + (size_t)j * sa * vec;
      if (use_prec) {
        if ((rc = prec(Vj, Z, sa))) return rc;
        if ((rc = op(Z, W, sa))) return rc;
      } else if ((rc = op(Vj, W, sa))) {
        return rc;
      }
      ++iters;
      const int k = (j + 1) * sa;
      std::vector<cd> hs((size_t)k * sa, cd(0.0)), hp;
      for (int pass = 0; pass < 2; ++pass) {
        if ((rc = gram(V, k, W, sa, hp))) return rc;
        HIPCHK(h, ems::launch_baxpy(V, k, Hd, sa, n, W, -1.0, 1.0, st));
        for (size_t e = 0; e < hs.size(); ++e) hs[e] += hp[e];
      }
      std::vector<cd> T;
      if ((rc = cholqr2(W, sa, V + (size_t)k * vec, T, ok))) return rc;
      if (!ok) {
        T.assign((size_t)sa * sa, cd(0.0));
        breakdown = true;
      }
      // new columns js .. js + s - 1: rows 0 .. k + s - 1
      for (int q = 0; q < sa; ++q) {
        const int c = j * sa + q;
        std::vector<cd> col((size_t)c + sa + 1, cd(0.0));
        for (int i = 0; i < k; ++i) col[i] = hs[(size_t)i * sa + q];
        for (int i = 0; i <= q; ++i) col[(size_t)k + i] = T[(size_t)i * sa + q];
        for (int cp = 0; cp < c; ++cp)
          for (int t = 0; t < sa; ++t) {
            const int row = cp + sa - t;  // rotation of rows (row - 1, row)
            rotate(rcs[(size_t)cp * sa + t], rsn[(size_t)cp * sa + t], col[row - 1], col[row]);
          }
        for (int t = 0; t < sa; ++t) {
          const int row = c + sa - t;
          const cd a = col[row - 1], bb = col[row];
          const double den = std::hypot(std::abs(a), std::abs(bb));
          cd cs = 1.0, sn = 0.0;
          if (den > 0) {
            cs = std::conj(a) / den;
            sn = std::conj(bb) / den;
          }
          rcs[(size_t)c * sa + t] = cs;
          rsn[(size_t)c * sa + t] = sn;
          rotate(cs, sn, col[row - 1], col[row]);
          col[row] = 0.0;
          for (int r = 0; r < sa; ++r)
            rotate(cs, sn, Gr[(size_t)(row - 1) * sa + r], Gr[(size_t)row * sa + r]);
        }
        Hc.push_back(std::move(col));
      }
      J = j + 1;
      // residual estimates: rows (j + 1) s .. (j + 2) s - 1 of the rotated RHS
      double emax = 0.0;
      for (int r = 0; r < sa; ++r) {
        double e2 = 0.0;
        for (int i = k; i < k + sa; ++i) e2 += std::norm(Gr[(size_t)i * sa + r]);
        emax = std::max(emax, std::sqrt(e2) / bnorm[act[r]]);
      }
      h->hist.push_back(emax);
      if (h->progress && h->progress_every > 0 && (int)h->hist.size() % h->progress_every == 0)
        h->progress((int32_t)h->hist.size(), emax, h->progress_user);
      if (emax <= tol || breakdown) break;
    }
    // Y = R^{-1} G (upper triangular, J s columns), then x += M^{-1} V Y
    const int m = J * sa;
    std::vector<cd> Y((size_t)m * sa, cd(0.0));
    for (int r = 0; r < sa; ++r)
      for (int i = m - 1; i >= 0; --i) {
        cd v = Gr[(size_t)i * sa + r];
        for (int l = i + 1; l < m; ++l) v -= Hc[l][i] * Y[(size_t)l * sa + r];
        const cd d = Hc[i][i];
        Y[(size_t)i * sa + r] = std::abs(d) > 0 ? v / d : cd(0.0);
      }
    {
      const auto y = to_dev_layout(Y);
      HIPCHK(h, hipMemcpyAsync(Hd, y.data(), sizeof(double2) * y.size(), hipMemcpyHostToDevice, st));
      HIPCHK(h, ems::launch_baxpy(V, m, Hd, sa, n, W, 1.0, 0.0, st));
      const double2 *upd = W;
      if (use_prec) {
        if ((rc = prec(W, Z, sa))) return rc;
        upd = Z;
      }
      for (int a = 0; a < sa; ++a)
        HIPCHK(h, ems::launch_axpy(x + (size_t)act[a] * vec, upd + (size_t)a * vec, n, 1.0, st));
      HIPCHK(h, hipStreamSynchronize(st));
    }
  }
  return EMS_OK;
}

}  // namespace

namespace {

// Euclidean norms of nrhs stacked vectors (device) into host memory.
int norms(ems_handle *h, const double2 *v, int nrhs, std::vector<double> &out, hipStream_t st) {
  // result (8 doubles, aligned for the partials) + kRedBlocks complex partials
  int rc = ensure_red(h, sizeof(double) * 8 + sizeof(double2) * ems::kRedBlocks);
  if (rc) return rc;
  double *d_nrm = reinterpret_cast<double *>(h->d_red);
  double *scratch = d_nrm + 8;
  out.assign(nrhs, 0.0);
  for (int r = 0; r < nrhs; ++r) {
    HIPCHK(h, ems::launch_norm2(v + (size_t)r * h->ncoef, h->ncoef, d_nrm, scratch, st));
    HIPCHK(h, hipMemcpyAsync(&out[r], d_nrm, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
  }
  return EMS_OK;
}

// R = b - A x for nrhs systems.
template <typename Op>
int residual(ems_handle *h, Op op, const double2 *x, const double2 *b, double2 *R, int nrhs,
             hipStream_t st) {
  int rc = op(x, R);
  if (rc) return rc;
  for (int r = 0; r < nrhs; ++r) {
    const size_t o = (size_t)r * h->ncoef;
    HIPCHK(h, ems::launch_scale(R + o, h->ncoef, -1.0, st));
    HIPCHK(h, ems::launch_axpy(R + o, b + o, h->ncoef, 1.0, st));
  }
  return EMS_OK;
}

// Buffers of the mixed-precision refinement (residual and correction).
int ensure_ir(ems_handle *h, int nrhs) {
  const size_t bytes = sizeof(double2) * (size_t)h->ncoef * nrhs;
  if (h->ir_bytes >= bytes) return EMS_OK;
  dfree(h->d_irR);
  dfree(h->d_irD);
  h->ir_bytes = 0;
  HIPCHK(h, hipMalloc(&h->d_irR, bytes));
  HIPCHK(h, hipMalloc(&h->d_irD, bytes));
  h->ir_bytes = bytes;
  return EMS_OK;
}

// GMRES on A (adjoint = false) or A^H, FP64 or mixed (FP32 contractions in an
// inner GMRES on the residual equation, FP64 outer residual and update), with
// or without the cluster block-Jacobi right preconditioner (for A^H its
// adjoint: the conjugate transpose of every block, applied to the clusters).
int solve_impl(ems_handle *h, const void *b, void *x, int32_t nrhs, const ems_solver_opts *o,
               ems_solve_info *info, ems_stream_t stream, bool adjoint) {
  if (!h || !b || !x || !o || nrhs <= 0) return fail(h, EMS_ERR_ARG, "bad solve arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  if (!(o->tol > 0) || o->maxit <= 0) return fail(h, EMS_ERR_ARG, "need tol > 0 and maxit > 0");
  if (o->precision != 0 && o->precision != 1) return fail(h, EMS_ERR_ARG, "precision must be 0 or 1");
  if (o->precond != 0 && o->precond != 1) return fail(h, EMS_ERR_ARG, "precond must be 0 or 1");
  if (o->block != 0 && o->block != 1) return fail(h, EMS_ERR_ARG, "block must be 0 or 1");
  if (o->block && o->precision != 0)
    return fail(h, EMS_ERR_ARG, "block GMRES runs in FP64 (precision 0)");
  hipStream_t st = (hipStream_t)stream;
  const auto t0 = std::chrono::steady_clock::now();
  const size_t vec = (size_t)h->ncoef;
  double2 *X = (double2 *)x;
  const double2 *B = (const double2 *)b;
  int rc;
  h->hist.clear();
  h->reorth = 0;
  const bool use_prec = o->precond == 1;
  if (use_prec && (rc = build_precond(h, st))) return rc;
  HIPCHK(h, hipMemsetAsync(X, 0, sizeof(double2) * vec * nrhs, st));
  int restart = o->restart;
  if (restart <= 0) {
    // as long as the basis fits in half of the free device memory
    size_t fr = 0, tot = 0;
    HIPCHK(h, hipMemGetInfo(&fr, &tot));
    const size_t have = fr / 2 + h->V_bytes;
    const size_t per = sizeof(double2) * vec * nrhs;
    restart = (int)std::max<size_t>(20, std::min<size_t>(5000, have / per - 1));
  }
  int iters = 0, outer = 1;
  double relres = 0;
  // the operator never aliases GMRES's internal buffers: it reads a basis
  // vector, a preconditioned vector or the iterate and writes the work vector
  auto op64 = [&](const double2 *in, double2 *out) {
    return apply_impl(h, in, out, nrhs, EMS_APPLY_ALL, adjoint, st);
  };
  auto op32 = [&](const double2 *in, double2 *out) {
    return apply_impl(h, in, out, nrhs, EMS_APPLY_ALL | EMS_MIXED, adjoint, st);
  };
  auto pc = [&](const double2 *in, double2 *out) {
    ems::ProfScope ps(h, "precond_apply", st, 8.0 * (double)h->pc_store * nrhs);
    HIPCHK(h, ems::launch_pc_apply(h, in, out, nrhs, adjoint, st));
    return EMS_OK;
  };
  if (o->block) {
    // groups of up to 64 right-hand sides, each one block Krylov space
    int mblk = o->restart;
    if (mblk <= 0) {
      size_t fr = 0, tot = 0;
      HIPCHK(h, hipMemGetInfo(&fr, &tot));
      const size_t have = fr / 2 + h->V_bytes;
      const int sg = std::min<int>(nrhs, 64);
      const size_t per = sizeof(double2) * vec * sg;
      // device basis from free memory; at most 8192 basis columns per cycle
      // (the host keeps the rotated block Hessenberg, about 0.5 GB there)
      mblk = (int)std::max<size_t>(2, std::min<size_t>(8192 / sg, have / per - 1));
    }
    restart = mblk;
    relres = 0.0;
    for (int g0 = 0; g0 < nrhs; g0 += 64) {
      const int sg = std::min(64, nrhs - g0);
      auto opb = [&](const double2 *in, double2 *out, int cnt) {
        return apply_impl(h, in, out, cnt, EMS_APPLY_ALL, adjoint, st);
      };
      auto pcb = [&](const double2 *in, double2 *out, int cnt) {
        ems::ProfScope ps(h, "precond_apply", st, 8.0 * (double)h->pc_store * cnt);
        HIPCHK(h, ems::launch_pc_apply(h, in, out, cnt, adjoint, st));
        return EMS_OK;
      };
      int it = 0;
      double rr = 0.0;
      rc = block_gmres_run(h, opb, pcb, use_prec, B + (size_t)g0 * vec, X + (size_t)g0 * vec, sg,
                           o->tol, mblk, o->maxit, st, it, rr);
      if (rc) return rc;
      iters += it;
      relres = std::max(relres, rr);
    }
  } else if (o->precision == 0) {
    std::vector<double> bn;
    rc = gmres_run(h, op64, pc, use_prec, B, X, nrhs, o->tol, restart, o->maxit, true, st, iters,
                   relres, bn, 1.0);
    if (rc) return rc;
  } else {
    if ((rc = ensure_ir(h, nrhs))) return rc;
    double2 *R = h->d_irR, *D = h->d_irD;
    const double itol = o->inner_tol > 0 ? o->inner_tol : 1e-3;
    std::vector<double> bn, rn;
    if ((rc = norms(h, B, nrhs, bn, st))) return rc;
    outer = 0;
    while (true) {
      if ((rc = residual(h, op64, X, B, R, nrhs, st))) return rc;
      if ((rc = norms(h, R, nrhs, rn, st))) return rc;
      relres = 0;
      double rmax = 0, bmax = 0;
      for (int r = 0; r < nrhs; ++r) {
        if (bn[r] > 0) relres = std::max(relres, rn[r] / bn[r]);
        rmax = std::max(rmax, rn[r]);
        bmax = std::max(bmax, bn[r]);
      }
      if (relres <= o->tol || iters >= o->maxit || outer >= 50) break;
      ++outer;
      int it = 0;
      double rr = 0;
      std::vector<double> tmp;
      HIPCHK(h, hipMemsetAsync(D, 0, sizeof(double2) * vec * nrhs, st));
      // the inner solve needs no more than the factor still missing
      const double need = std::max(itol, 0.5 * o->tol / std::max(relres, 1e-300));
      // complex64 basis while the inner tolerance stays above 1e-5
      rc = gmres_run(h, op32, pc, use_prec, R, D, nrhs, need, restart, o->maxit - iters, true, st,
                     it, rr, tmp, relres, 200, need >= 1e-5);
      if (rc) return rc;
      iters += it;
      for (int r = 0; r < nrhs; ++r)
        HIPCHK(h, ems::launch_axpy(X + r * vec, D + r * vec, h->ncoef, 1.0, st));
    }
  }
  HIPCHK(h, hipStreamSynchronize(st));
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  const bool conv = relres <= o->tol * 1.0000001;
  if (info) {
    info->iters = iters;
    info->outer_iters = outer;
    info->relres = relres;
    info->converged = conv ? 1 : 0;
    info->seconds = secs;
    info->restart = restart;
    info->reorth = h->reorth;
    info->precond_seconds = use_prec ? h->pc_setup_s : 0.0;
  }
  return conv ? EMS_OK : EMS_NOT_CONVERGED;
}

}  // namespace

extern "C" int ems_set_exponentials(ems_handle *h, int32_t tabulate) {
  if (!h) return EMS_ERR_ARG;
  if (tabulate != 0 && tabulate != 1) return fail(h, EMS_ERR_ARG, "tabulate must be 0 or 1");
  h->somm_tab = tabulate == 1;
  return EMS_OK;
}

extern "C" int ems_set_precond(ems_handle *h, int32_t max_unknowns) {
  if (!h) return EMS_ERR_ARG;
  if (max_unknowns == 0) max_unknowns = 512;
  if (max_unknowns < 1 || max_unknowns > 512)
    return fail(h, EMS_ERR_ARG, "cluster size must be in [1, 512] unknowns");
  if (h->pc_cap != max_unknowns) {
    h->pc_cap = max_unknowns;
    dfree(h->d_pc_inv);
    h->pc_built = false;
  }
  return EMS_OK;
}

extern "C" int ems_precond_apply(ems_handle *h, const void *x, void *y, int32_t nrhs,
                                 int32_t adjoint, int32_t *clusters, int32_t *max_rows,
                                 double *setup_s, ems_stream_t stream) {
  if (!h || !x || !y || nrhs <= 0 || x == y) return fail(h, EMS_ERR_ARG, "bad preconditioner arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  hipStream_t st = (hipStream_t)stream;
  int rc = build_precond(h, st);
  if (rc) return rc;
  HIPCHK(h, ems::launch_pc_apply(h, (const double2 *)x, (double2 *)y, nrhs, adjoint != 0, st));
  if (clusters) *clusters = h->pc_nc;
  if (max_rows) *max_rows = h->pc_bmax;
  if (setup_s) *setup_s = h->pc_setup_s;
  return EMS_OK;
}

extern "C" int ems_set_progress(ems_handle *h, ems_progress_fn fn, int32_t every, void *user) {
  if (!h || (fn && every <= 0)) return fail(h, EMS_ERR_ARG, "progress needs every > 0");
  h->progress = fn;
  h->progress_every = fn ? every : 0;
  h->progress_user = user;
  return EMS_OK;
}

extern "C" int ems_solve_history(const ems_handle *h, double *out, int32_t cap, int32_t *count) {
  if (!h || !count || cap < 0 || (cap > 0 && !out)) return EMS_ERR_ARG;
  *count = (int32_t)h->hist.size();
  for (int i = 0; i < cap && i < (int)h->hist.size(); ++i) out[i] = h->hist[i];
  return EMS_OK;
}

extern "C" int ems_solve(ems_handle *h, const void *b, void *x, int32_t nrhs,
                         const ems_solver_opts *o, ems_solve_info *info, ems_stream_t stream) {
  return solve_impl(h, b, x, nrhs, o, info, stream, false);
}

extern "C" int ems_solve_adjoint(ems_handle *h, const void *b, void *x, int32_t nrhs,
                                 const ems_solver_opts *o, ems_solve_info *info,
                                 ems_stream_t stream) {
  return solve_impl(h, b, x, nrhs, o, info, stream, true);
}

namespace {

// Receivers must lie in the host layer (y < 0) and outside every enclosing disk.
// Receivers: finite, off the interface, in the host outside every enclosing
// disk, or (when substrate is non-null) in the substrate, counted there.
int check_receivers(ems_handle *h, const double *pts, int npts, hipStream_t st,
                    double *depth = nullptr, int *substrate = nullptr) {
  std::vector<double> hp(2 * (size_t)npts);
  HIPCHK(h, hipMemcpyAsync(hp.data(), pts, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  if (depth) *depth = HUGE_VAL;
  if (substrate) *substrate = 0;
  for (int i = 0; i < npts; ++i) {
    const double x = hp[2 * i], y = hp[2 * i + 1];
    if (!std::isfinite(x) || !std::isfinite(y)) return fail(h, EMS_ERR_NUMERIC, "non-finite receiver");
    if (depth) *depth = std::min(*depth, -y);
    if (substrate && y > 0) {
      ++*substrate;
      continue;
    }
    if (!(y < 0))
      return fail(h, EMS_ERR_GEOMETRY,
                  substrate ? "receiver on the interface (y = 0)"
                            : "receiver not in the host layer (y < 0)");
    for (int m = 0; m < h->n; ++m) {
      const double dx = x - h->xy[2 * m], dy = y - h->xy[2 * m + 1];
      if (dx * dx + dy * dy <= h->R[m] * h->R[m])
        return fail(h, EMS_ERR_GEOMETRY,
                    "receiver " + std::to_string(i) + " inside the enclosing disk of particle " +
                        std::to_string(m));
    }
  }
  return EMS_OK;
}

// Depth-truncation ranges with receivers at depth dr at the other end of
// the pairs.  Receivers shallower than every particle see more of each
// node's particles than the operator's pairs do; the ranges for them are
// formed on the host from the handle's node table and cached per depth.
// *kc, *jr stay nullptr (the build's ranges) when dr is not shallower.
int field_cuts(ems_handle *h, double dr, const int **kc, const int **jr) {
  *kc = nullptr;
  *jr = nullptr;
  if (!h->d_kcut || !(dr < h->depth_min)) return EMS_OK;
  if (h->cut_f_depth != dr) {
    ems::DepthCuts dc;
    ems::depth_cuts(h->nodes, h->md, h->xy, h->pmax, h->somm.depth_cut, dr, dc);
    int rc;
    if ((rc = upload(h, h->d_kcut_f, dc.kcut.data(), dc.kcut.size()))) return rc;
    if ((rc = upload(h, h->d_jr_f, dc.jr.data(), dc.jr.size()))) return rc;
    h->cut_f_depth = dr;
  }
  *kc = h->d_kcut_f;
  *jr = h->d_jr_f;
  return EMS_OK;
}

}  // namespace

extern "C" int ems_eval_scattered(ems_handle *h, const void *gamma, int32_t nrhs, int32_t npts,
                                  const double *pts, void *u, ems_stream_t stream) {
  if (!h || !gamma || !pts || !u || nrhs <= 0 || npts <= 0)
    return fail(h, EMS_ERR_ARG, "bad field arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  hipStream_t st = (hipStream_t)stream;
  double dr = 0.0;
  int nsub = 0;
  int rc = check_receivers(h, pts, npts, st, &dr, &nsub);
  if (rc) return rc;
  if ((rc = ensure_ws(h, nrhs))) return rc;
  const int *kc = nullptr, *jr = nullptr;
  if ((rc = field_cuts(h, dr, &kc, &jr))) return rc;
  const double2 *g = (const double2 *)gamma;
  double2 *uo = (double2 *)u;
  {
    ems::ProfScope ps(h, "field_direct", st);
    HIPCHK(h, ems::launch_field_direct(h, g, nrhs, npts, pts, uo, st));
  }
  HIPCHK(h, ems::launch_somm_aggregate(h, g, nrhs, false, false, st, kc));
  HIPCHK(h, ems::launch_somm_reflect(h, nrhs, false, st));
  {
    ems::ProfScope ps(h, "field_refl", st);
    HIPCHK(h, ems::launch_field_refl(h, nrhs, npts, pts, uo, st));
  }
  if (nsub > 0) {
    // substrate receivers: the same aggregate through T(xi) instead of R(xi)
    HIPCHK(h, ems::launch_somm_reflect(h, nrhs, false, st, true));
    ems::ProfScope ps(h, "field_trans", st);
    HIPCHK(h, ems::launch_field_trans(h, nrhs, npts, pts, uo, st));
  }
  return EMS_OK;
}

extern "C" int ems_eval_scattered_adjoint(ems_handle *h, const void *res, int32_t nrhs,
                                          int32_t npts, const double *pts, void *g,
                                          ems_stream_t stream) {
  if (!h || !res || !pts || !g || nrhs <= 0 || npts <= 0)
    return fail(h, EMS_ERR_ARG, "bad field arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  hipStream_t st = (hipStream_t)stream;
  double dr = 0.0;
  int rc = check_receivers(h, pts, npts, st, &dr);
  if (rc) return rc;
  if ((rc = ensure_ws(h, nrhs))) return rc;
  const int *kc = nullptr, *jr = nullptr;
  if ((rc = field_cuts(h, dr, &kc, &jr))) return rc;
  const double2 *rs = (const double2 *)res;
  {
    ems::ProfScope ps(h, "field_direct_adjoint", st);
    HIPCHK(h, ems::launch_field_direct_adjoint(h, rs, nrhs, npts, pts, h->d_free, st));
  }
  {
    ems::ProfScope ps(h, "field_refl_adjoint", st);
    HIPCHK(h, ems::launch_field_refl_adjoint(h, rs, nrhs, npts, pts, st));
  }
  HIPCHK(h, ems::launch_somm_reflect(h, nrhs, true, st));
  HIPCHK(h, ems::launch_somm_disaggregate(h, nrhs, true, false, st, jr));
  HIPCHK(h, ems::launch_combine(h, nullptr, (double2 *)g, nrhs, EMS_PART_FREE | EMS_PART_REFL,
                                true, false, st));
  return EMS_OK;
}

namespace {

// The operator with orders p + 1 and S = I on the same geometry, media,
// Sommerfeld rule kind and FMM settings: its free + reflected parts give the
// order-(p + 1) incoming and adjoint expansions the centre gradient needs,
// its plane-wave right-hand side the raw local coefficients.  Built once per
// build of the parent; the exponential tables are left out (the vector-ALU
// contractions form them on the fly).
int build_ext(ems_handle *h, hipStream_t st) {
  if (h->pmax + 1 > ems::kMaxP)
    return fail(h, EMS_ERR_UNIMPLEMENTED, "gradient needs truncation orders below 16");
  ems_handle *e = nullptr;
  int rc = ems_create(&e);
  if (rc) return fail(h, rc, "cannot create the extended operator");
  e->md = h->md;
  e->have_media = true;
  std::vector<int32_t> pe(h->n);
  for (int i = 0; i < h->n; ++i) pe[i] = h->p[i] + 1;
  rc = ems_set_particles(e, h->n, h->xy.data(), h->R.data(), pe.data());
  if (rc == EMS_OK) {
    std::vector<int64_t> so(h->n + 1, 0);
    for (int i = 0; i < h->n; ++i) so[i + 1] = so[i] + (int64_t)(4 * pe[i] + 2) * (4 * pe[i] + 2);
    std::vector<double> S(2 * (size_t)so[h->n], 0.0);
    for (int i = 0; i < h->n; ++i) {
      const int64_t K = 4 * pe[i] + 2;
      for (int64_t k = 0; k < K; ++k) S[2 * (size_t)(so[i] + k * K + k)] = 1.0;
    }
    rc = ems_set_smatrices(e, S.data(), so.data());
  }
  if (rc == EMS_OK) {
    e->somm = h->somm;
    e->fmm_mode = h->fmm_mode;
    e->fmm_leaf = h->fmm_leaf;
    e->fmm_top = h->fmm_top;
    e->fmm_digits = h->fmm_digits;
    e->etab_budget_gb = 0.0;
    rc = ems_build(e, st);
  }
  if (rc) {
    const std::string msg = "extended operator: " + std::string(e->err);
    ems_destroy(e);
    return fail(h, rc, msg);
  }
  h->ext = e;
  return EMS_OK;
}

}  // namespace

extern "C" int ems_param_vjp(ems_handle *h, const ems_plane_wave *waves, int32_t nrhs,
                             const void *gamma, const void *lam, int32_t npts, const double *pts,
                             const void *res, double *dxy, double *dlame, ems_stream_t stream) {
  if (!h || !waves || !gamma || !lam || !pts || !res || !dxy || !dlame || nrhs <= 0 || npts <= 0)
    return fail(h, EMS_ERR_ARG, "bad gradient arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  for (int r = 0; r < nrhs; ++r)
    if (waves[r].wave != 0 && waves[r].wave != 1)
      return fail(h, EMS_ERR_UNIMPLEMENTED,
                  "gradient for waves sent from the substrate (dT/dtheta) is not built");
  hipStream_t st = (hipStream_t)stream;
  double dr = 0.0;
  int rc = check_receivers(h, pts, npts, st, &dr);
  if (rc) return rc;
  const int *kc = nullptr, *jr = nullptr;
  if ((rc = field_cuts(h, dr, &kc, &jr))) return rc;
  if (!h->ext && (rc = build_ext(h, st))) return rc;
  ems_handle *E = h->ext;
  if ((rc = ensure_ws(h, nrhs))) return rc;
  const size_t nh = (size_t)nrhs * h->ncoef, ne = (size_t)nrhs * E->ncoef;
  const size_t nq = (size_t)nrhs * 2 * h->q;
  constexpr int kBlocks = 256;
  double2 *buf = nullptr;
  HIPCHK(h, hipMalloc(&buf, sizeof(double2) * (2 * nh + 6 * ne + 2 * nq) + sizeof(double) * 8 * kBlocks));
  double2 *mu = buf, *a0dR = mu + nh, *gpad = a0dR + nh, *mpad = gpad + ne, *ae = mpad + ne,
          *ze = ae + ne, *fe = ze + ne, *a0e = fe + ne, *Ig = a0e + ne, *Lam = Ig + nq;
  double *part = reinterpret_cast<double *>(Lam + nq);
  const double2 *G = (const double2 *)gamma;
  auto run = [&]() -> int {
    // mu = S^H lambda
    HIPCHK(h, ems::launch_s_apply(h, (const double2 *)lam, mu, nrhs, true, st));
    HIPCHK(h, ems::launch_repack(h, E, G, gpad, nrhs, st));
    HIPCHK(h, ems::launch_repack(h, E, mu, mpad, nrhs, st));
    int r2 = apply_impl(E, gpad, ae, nrhs, EMS_PART_FREE | EMS_PART_REFL, false, st);
    if (r2) return fail(h, r2, std::string("extended apply: ") + E->err);
    r2 = apply_impl(E, mpad, ze, nrhs, EMS_PART_FREE | EMS_PART_REFL, true, st);
    if (r2) return fail(h, r2, std::string("extended adjoint apply: ") + E->err);
    r2 = ems_eval_scattered_adjoint(E, res, nrhs, npts, pts, fe, st);
    if (r2) return fail(h, r2, std::string("extended field adjoint: ") + E->err);
    r2 = ems_incident(E, waves, nrhs, a0e, st);
    if (r2) return fail(h, r2, std::string("extended incident: ") + E->err);
    HIPCHK(h, ems::launch_grad_centres(h, E, G, mu, ae, a0e, fe, ze, nrhs, dxy, st));
    // Lame parameters: node term
    // Ig meets the receivers' reflected terms as well: their depth ranges
    HIPCHK(h, ems::launch_somm_aggregate(h, G, nrhs, false, false, st, kc));
    HIPCHK(h, ems::launch_lame_ig(h, nrhs, Ig, st));
    HIPCHK(h, ems::launch_somm_aggregate(h, mu, nrhs, true, false, st));
    HIPCHK(h, ems::launch_lame_lam(h, nrhs, Lam, false, st));
    HIPCHK(h, ems::launch_field_refl_adjoint(h, (const double2 *)res, nrhs, npts, pts, st));
    HIPCHK(h, ems::launch_lame_lam(h, nrhs, Lam, true, st));
    HIPCHK(h, ems::launch_lame_reduce(h, nrhs, Ig, Lam, part, kBlocks, st));
    // right-hand-side term: the reflected plane wave with dR(xi0) in place of R(xi0)
    const cd I(0.0, 1.0);
    std::vector<double2> pw[2];
    for (int th = 0; th < 2; ++th) pw[th].resize(7 * (size_t)nrhs);
    for (int r = 0; r < nrhs; ++r) {
      const int wv = waves[r].wave;
      const double k = wv == 0 ? h->md.kp : h->md.ks;
      const double xi0 = k * std::sin(waves[r].angle);
      const cd A = 1.0 / (I * k);
      const cd Ap = wv == 0 ? A : 0.0, As = wv == 1 ? A : 0.0;
      cd R0[4], dR0[8];
      if (ems::reflection_deriv(cd(xi0, 0.0), h->md, R0, dR0))
        return fail(h, EMS_ERR_NUMERIC, "singular interface system at the incident wavenumber");
      const cd s1 = ems::branch_s(cd(xi0, 0.0), h->md.kp), s2 = ems::branch_s(cd(xi0, 0.0), h->md.ks);
      for (int th = 0; th < 2; ++th) {
        const cd *D = dR0 + 4 * th;
        const cd v[7] = {cd(xi0, 0.0), s1, s2, 0.0, 0.0, D[0] * Ap + D[1] * As, D[2] * Ap + D[3] * As};
        for (int k2 = 0; k2 < 7; ++k2)
          pw[th][7 * (size_t)r + k2] = make_double2(v[k2].real(), v[k2].imag());
      }
    }
    double2 *dpw = Ig;  // Ig is consumed by the node reduction above; reuse as upload space
    for (int th = 0; th < 2; ++th) {
      HIPCHK(h, hipMemcpyAsync(dpw, pw[th].data(), pw[th].size() * sizeof(double2),
                               hipMemcpyHostToDevice, st));
      HIPCHK(h, ems::launch_incident_pw(h, dpw, nrhs, a0dR, st));
      HIPCHK(h, ems::launch_re_dot((int64_t)nh, mu, a0dR, part + (2 + th) * kBlocks, kBlocks, st));
      HIPCHK(h, hipStreamSynchronize(st));  // dpw is rewritten for the next parameter
    }
    std::vector<double> hp(4 * kBlocks);
    HIPCHK(h, hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    double s[2] = {0.0, 0.0};
    for (int b = 0; b < kBlocks; ++b) {
      s[0] += hp[2 * b];
      s[1] += hp[2 * b + 1];
    }
    for (int b = 0; b < kBlocks; ++b) {
      s[0] += hp[2 * kBlocks + b];
      s[1] += hp[3 * kBlocks + b];
    }
    dlame[0] = s[0];
    dlame[1] = s[1];
    return EMS_OK;
  };
  rc = run();
  (void)hipStreamSynchronize(st);
  (void)hipFree(buf);
  return rc;
}

extern "C" int ems_autotune(ems_handle *h, int32_t nrhs, int32_t *chosen, ems_stream_t stream) {
  if (!h || nrhs <= 0) return fail(h, EMS_ERR_ARG, "bad autotune arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  if (chosen)
    for (int k = 0; k < 8; ++k) chosen[k] = 0;
  if (!ems::somm_mfma_ready(h, false)) return EMS_OK;  // the vector-ALU kernels run
  hipStream_t st = (hipStream_t)stream;
  int rc = ensure_ws(h, nrhs);
  if (rc) return rc;
  const size_t vec = sizeof(double2) * (size_t)nrhs * h->ncoef;
  if ((rc = ensure_tmp(h, vec))) return rc;
  // inputs of the timed launches: zero coefficients and node amplitudes
  HIPCHK(h, hipMemsetAsync(h->d_tmp, 0, vec, st));
  HIPCHK(h, hipMemsetAsync(h->d_refl, 0, sizeof(double2) * (size_t)nrhs * 2 * h->q, st));
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  const int batched = nrhs > 1 ? 1 : 0;
  for (int kernel = 0; kernel < 2; ++kernel)
    for (int prec = 0; prec < 2; ++prec) {
      if (prec == 1 && !ems::somm_mfma_fp32(h)) continue;
      float best = 1e30f;
      int bi = -1;
      for (int idx = 0; idx < 4; ++idx) {
        int nt = 0, rb = 0;
        ems::mfma_candidate(kernel, prec, idx, &nt, &rb);
        if (rb > 1 && nrhs == 1) continue;  // batched shapes only pay with several RHS
        float tmin = 1e30f;
        for (int rep = 0; rep < 5; ++rep) {
          HIPCHK(h, hipEventRecord(e0, st));
          hipError_t e = kernel == 0
                             ? ems::launch_somm_aggregate_mfma(h, h->d_tmp, nrhs, prec, idx, st)
                             : ems::launch_somm_disaggregate_mfma(h, nrhs, prec, idx, st);
          HIPCHK(h, e);
          HIPCHK(h, hipEventRecord(e1, st));
          HIPCHK(h, hipEventSynchronize(e1));
          float ms = 0.f;
          HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
          if (rep > 0) tmin = std::min(tmin, ms);  // the first launch warms caches and code
        }
        if (tmin < best) {
          best = tmin;
          bi = idx;
        }
      }
      h->mfma_cfg[kernel][prec][batched] = bi;
      if (chosen) {
        int nt = 0, rb = 0;
        ems::mfma_candidate(kernel, prec, bi, &nt, &rb);
        chosen[4 * kernel + 2 * prec] = nt;
        chosen[4 * kernel + 2 * prec + 1] = rb;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return EMS_OK;
}

// ---------------------------------------------------------------------------
// Operator apply without allocation: the per-call workspace of ems_apply
// (Sommerfeld aggregate partials and reflected amplitudes, disaggregate
// partials, the free-space output, FMM expansions and task-group partials)
// lives in one static device array per GPU instead of handle-owned
// allocations.
namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) double2 scratch[kScratchBytes / sizeof(double2)];

std::mutex g_scratch_mu;
std::map<int, double2 *> g_scratch_ptr;  // device -> address of that device's array

__global__ void scratch_fill_zero(double2 *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_double2(0.0, 0.0);
}

// Address of the current device's array, looked up once per device.
int scratch_address(ems_handle *h, double2 **out) {
  int dev = 0;
  HIPCHK(h, hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(h, EMS_ERR_HIP,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    it = g_scratch_ptr.emplace(dev, reinterpret_cast<double2 *>(p)).first;
  }
  *out = it->second;
  return EMS_OK;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" int ems_apply_noalloc(ems_handle *h, const void *x, void *y, int32_t nrhs,
                                 int32_t flags, ems_stream_t stream) {
  if (!h || !x || !y || nrhs <= 0 || x == y) return fail(h, EMS_ERR_ARG, "bad apply arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  if (h->prof)
    return fail(h, EMS_ERR_STATE, "kernel profiling creates events: switch it off for this call");
  double2 *base = nullptr;
  int rc = scratch_address(h, &base);
  if (rc) return rc;
  // workspace layout: the chunk counts of ems_apply, halved until it fits
  const size_t nc = (size_t)h->ncoef, c16 = sizeof(double2);
  const int node_tiles = (h->q + 255) / 256, part_tiles = (h->n + 255) / 256;
  int agg = std::max(1, std::min(std::max(1, h->n / 8),
                                 (4096 + 2 * nrhs * node_tiles - 1) / (2 * nrhs * node_tiles)));
  int dis = std::max(1, std::min(std::max(1, h->q / 32),
                                 (ems::kDisChunkTarget + 2 * nrhs * part_tiles - 1) / (2 * nrhs * part_tiles)));
  auto need = [&](int a, int d, size_t *o) {
    size_t t = 0;
    o[0] = t; t += align256(c16 * nrhs * 2 * (size_t)a * h->q);   // aggregate partials
    o[1] = t; t += align256(c16 * nrhs * 2 * (size_t)h->q);       // reflected amplitudes
    o[2] = t; t += align256(c16 * nrhs * (size_t)d * nc);         // disaggregate partials
    o[3] = t; t += align256(c16 * nrhs * nc);                     // free-space output
    o[8] = t; t += align256(c16 * (h->d_xpad ? xpad_len(h, nrhs) : 0));  // padded coefficients
    o[9] = t; t += align256(c16 * (h->d_bpad ? bpad_len(h, nrhs) : 0));  // padded node operand
    o[4] = o[5] = o[6] = o[7] = t;
    if (h->fmm_on) {
      o[4] = t; t += align256(c16 * nrhs * (size_t)h->fmm.exp_len);
      o[5] = t; t += align256(c16 * nrhs * (size_t)h->fmm.exp_len);
      o[6] = t; t += align256(c16 * nrhs * (size_t)h->fmm.max_slots * ems::kFmmRows);
      o[7] = t; t += align256(c16 * nrhs * (size_t)h->fmm.m2l.part_len);
    }
    return t;
  };
  size_t o[10];
  size_t total = need(agg, dis, o);
  while (total > kScratchBytes && (dis > 1 || agg > 1)) {
    if (dis > 1) dis = (dis + 1) / 2;
    else agg = (agg + 1) / 2;
    total = need(agg, dis, o);
  }
  if (total > kScratchBytes)
    return fail(h, EMS_ERR_ARG,
                "apply workspace of " + std::to_string(total) + " bytes exceeds the " +
                    std::to_string(kScratchBytes) + "-byte static scratch (fewer right-hand sides)");
  hipStream_t st = (hipStream_t)stream;
  // whatever an earlier call left there: the partial sums start from zero
  hipLaunchKernelGGL(scratch_fill_zero, dim3(1024), dim3(256), 0, st, base,
                     (int64_t)(total / c16));
  HIPCHK(h, hipGetLastError());
  char *b = reinterpret_cast<char *>(base);
  double2 *sv[10] = {h->d_agg,  h->d_refl, h->d_dis,      h->d_free,     h->d_mult,
                     h->d_loc,  h->d_fmm_part, h->d_m2l_part, h->d_xpad, h->d_bpad};
  const int s_agg = h->agg_chunks, s_dis = h->dis_chunks, s_ws = h->ws_nrhs;
  h->d_agg = reinterpret_cast<double2 *>(b + o[0]);
  h->d_refl = reinterpret_cast<double2 *>(b + o[1]);
  h->d_dis = reinterpret_cast<double2 *>(b + o[2]);
  h->d_free = reinterpret_cast<double2 *>(b + o[3]);
  h->d_xpad = sv[8] ? reinterpret_cast<double2 *>(b + o[8]) : nullptr;
  h->d_bpad = sv[9] ? reinterpret_cast<double2 *>(b + o[9]) : nullptr;
  h->d_mult = h->fmm_on ? reinterpret_cast<double2 *>(b + o[4]) : nullptr;
  h->d_loc = h->fmm_on ? reinterpret_cast<double2 *>(b + o[5]) : nullptr;
  h->d_fmm_part = (h->fmm_on && h->fmm.max_slots > 0) ? reinterpret_cast<double2 *>(b + o[6])
                                                      : nullptr;
  h->d_m2l_part = (h->fmm_on && h->fmm.m2l.part_len > 0) ? reinterpret_cast<double2 *>(b + o[7])
                                                         : nullptr;
  h->agg_chunks = agg;
  h->dis_chunks = dis;
  h->ws_nrhs = nrhs;  // the workspace is in place: the apply sizes nothing
  rc = apply_impl(h, (const double2 *)x, (double2 *)y, nrhs, flags, false, st);
  h->d_agg = sv[0];
  h->d_refl = sv[1];
  h->d_dis = sv[2];
  h->d_free = sv[3];
  h->d_mult = sv[4];
  h->d_loc = sv[5];
  h->d_fmm_part = sv[6];
  h->d_m2l_part = sv[7];
  h->d_xpad = sv[8];
  h->d_bpad = sv[9];
  h->agg_chunks = s_agg;
  h->dis_chunks = s_dis;
  h->ws_nrhs = s_ws;
  return rc;
}

extern "C" int ems_apply_graph(ems_handle *h, const void *x, void *y, int32_t nrhs, int32_t flags,
                               int32_t adjoint, ems_stream_t stream) {
  if (!h || !x || !y || nrhs <= 0 || x == y) return fail(h, EMS_ERR_ARG, "bad apply arguments");
  if (!h->built) return fail(h, EMS_ERR_STATE, "ems_build first");
  hipStream_t st = (hipStream_t)stream;
  const auto key = std::make_tuple(x, y, (int)nrhs, (int)flags, adjoint ? 1 : 0);
  auto it = h->graphs.find(key);
  if (it == h->graphs.end() || it->second.second != h->ws_epoch) {
    if (it != h->graphs.end()) {
      (void)hipGraphExecDestroy(it->second.first);
      h->graphs.erase(it);
    }
    // eager apply: the result of this call, and every workspace sized before capture
    int rc = apply_impl(h, (const double2 *)x, (double2 *)y, nrhs, flags, adjoint != 0, st);
    if (rc) return rc;
    if (!h->cap_stream) {
      HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
      for (auto &e : h->cap_ev) HIPCHK(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    hipStream_t cs = st ? st : h->cap_stream;
    const uint64_t epoch = h->ws_epoch;
    const bool prof = h->prof;
    h->prof = false;
    HIPCHK(h, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    rc = apply_impl(h, (const double2 *)x, (double2 *)y, nrhs, flags, adjoint != 0, cs);
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &g);
    h->prof = prof;
    if (rc || ee != hipSuccess || h->ws_epoch != epoch) {
      if (g) (void)hipGraphDestroy(g);
      if (rc) return rc;
      return fail(h, EMS_ERR_HIP, "apply capture failed");
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(h, EMS_ERR_HIP, "graph instantiate failed");
    h->graphs[key] = std::make_pair(ex, epoch);
    return EMS_OK;
  }
  hipGraphExec_t ex = it->second.first;
  if (st) {
    HIPCHK(h, hipGraphLaunch(ex, st));
  } else {
    // join the null stream through events around the replay stream
    HIPCHK(h, hipEventRecord(h->cap_ev[0], st));
    HIPCHK(h, hipStreamWaitEvent(h->cap_stream, h->cap_ev[0], 0));
    HIPCHK(h, hipGraphLaunch(ex, h->cap_stream));
    HIPCHK(h, hipEventRecord(h->cap_ev[1], h->cap_stream));
    HIPCHK(h, hipStreamWaitEvent(st, h->cap_ev[1], 0));
  }
  return EMS_OK;
}
