// Internal declarations of the ems library: handle state, host set-up helpers
// and kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <map>
#include <tuple>
#include <vector>

#include "../../include/ems.h"

namespace ems {

using cd = std::complex<double>;

// Largest truncation order the kernels are built for: one wavefront (64
// lanes) holds the 2(2p+1) <= 62 coefficients of one particle.
constexpr int kMaxP = 16;
constexpr int kMaxModes = 2 * kMaxP + 1;
// blocks of the vector reductions (launch_norm2, launch_mdot): each writes
// kRedBlocks complex partials per reduced vector into its scratch argument
constexpr int kRedBlocks = 512;
// Split-K chunks of the Sommerfeld disaggregate over the nodes: about this
// many (particle tile, chunk, wave, right-hand side) slots per launch.  Every
// chunk writes one partial coefficient vector that the combine kernel reads
// back (13 chunks, 0.26 GB each way at 20000 particles in FP64).  With the
// 16-particle FP64 tile, 13 chunks cost the disaggregate nothing against 26
// and save the combine 0.08 ms; at 7 the disaggregate loses more than the
// combine gains (fewer, longer wavefronts over uneven depth-truncated node
// ranges).
constexpr int kDisChunkTarget = 2048;

struct Media {
  double lam_h, mu_h, rho_h, lam_b, mu_b, rho_b, omega;
  double kp, ks, kpb, ksb;
};

Media make_media(const ems_media &m);

// Sommerfeld node table (host copy).  xi and w are complex in general
// (the paper's tanh contour); real for the graded real-axis rule.
// Nodes of a branch-point substitution panel (xi = bp + d, d = +-u^2) keep
// bp and d so that s for the wavenumber |bp| is formed as sqrt(d (2 bp + d))
// without cancellation; bp = 0 marks an ordinary node.
struct NodeTable {
  std::vector<cd> xi, w;
  std::vector<double> bp, d;
  double t_max = 0.0;
};

struct SommerfeldSpec {
  int kind = 1;
  int q = 0;
  double t_max = 0.0;
  double delta = 0.5;
  double panel_scale = 1.0;
  int panel_order = 64;
  double tail_factor = 1.0;
  double depth_cut = 1e-26;  // depth truncation threshold (<= 0: none)
  std::vector<double> user;  // kind 2: [q][4]
};

// s(xi; k): decaying branch, Re s >= 0.  Real xi split by cases; complex xi
// with Im(k^2 - xi^2) >= 0 uses the principal root of k^2 - xi^2.
cd branch_s(cd xi, double k);

// Build the node table for the given cloud.
int build_nodes(const SommerfeldSpec &spec, const Media &md, const std::vector<double> &xy,
                const std::vector<int> &p, NodeTable &out, std::string &err);

// Depth truncation of the tabulated Sommerfeld contractions (setup.cpp):
// perm = particles by increasing depth; kcut[w q + j] = how many of them
// (in that order) node j of wave w keeps; jr[2 (w n + i)], jr[2 (w n + i) + 1]
// = the node range [lo, hi) that covers every node keeping the i-th of them.
struct DepthCuts {
  std::vector<int> perm, kcut, jr;
  double kept = 1.0;  // kept fraction of the (node, particle, wave) triples
};
// dother: depth of the shallowest point at the other end of a pair (the
// shallowest particle for the operator; receivers may be shallower).
void depth_cuts(const NodeTable &nodes, const Media &md, const std::vector<double> &xy, int pmax,
                double eps, double dother, DepthCuts &out);

// s(xi; k) for every wavenumber of the media at node (xi, bp, d):
// out = {s_p, s_s, s_pb, s_sb}.
void node_s(cd xi, double bp, double d, const Media &md, cd out[4]);

// 2x2 reflection R(xi) of upgoing P/S potentials at the welded interface,
// with the four branch values s given (node_s) or formed from xi.
int reflection(cd xi, const Media &md, cd R[4]);
int reflection_s(cd xi, const cd s[4], const Media &md, cd R[4]);
// The same system with the transmitted (substrate upgoing) potentials T too,
// and for waves sent from the substrate: Td = host downgoing (transmitted),
// Rb = substrate upgoing (reflected) potentials per unit downgoing P / S.
int reflect_transmit_s(cd xi, const cd s4[4], const Media &md, cd R[4], cd T[4]);
int from_substrate_s(cd xi, const cd s4[4], const Media &md, cd Td[4], cd Rb[4]);
int from_substrate(cd xi, const Media &md, cd Td[4], cd Rb[4]);
int reflection_deriv_s(cd xi, const cd s4[4], const Media &md, cd R[4], cd dR[8]);
int reflection_deriv(cd xi, const Media &md, cd R[4], cd dR[8]);

// Closed-form disk scattering matrix, row-major (4p+2)^2.
int disk_smatrix(const Media &md, double a, int p, int bc, std::vector<cd> &S);

// Free-space FMM plan (fmm.cpp): tree levels, expansion orders, near lists
// and the task lists of the batched Toeplitz kernel.
struct FmmLevel {
  std::vector<int> bx, by;
  int P[2] = {0, 0};
  int64_t off[2] = {0, 0};  // start of this level's expansions (per wave)
  double side = 0.0;
};

// One launch of the Toeplitz task kernel.  in_kind: 0 particle coefficients,
// 1 multipoles, 2 locals; out_kind: 1 multipoles, 2 locals, 3 free-part
// output.  Tasks with sgn = 2 read from the locals (L2L inside an M2L launch);
// sgn = -1 flips the odd symbol entries (L2P).
// Items of a launch are (output, 192-row chunk, task group): when a launch
// has few outputs their task lists are split into groups on separate
// wavefronts, each writing a partial chunk (slot) that a second kernel sums
// in a fixed order (red_* lists, one entry per (output, chunk)).
constexpr int kFmmRows = 192;
struct FmmLaunch {
  const char *name = "fmm";
  int gemm_level = -1;  // >= 0: the matrix-core M2L of that level (both waves), no tasks
  int in_kind = 0, out_kind = 0, accumulate = 0, nout = 0, max_in_P = 0, max_out_P = 0;
  double flops = 0.0;  // 8 (2 P_out + 1)(2 P_in + 1) summed over the tasks, per right-hand side
  std::vector<int> ptr, in_P, sym_L, sgn, out_P, item_out, item_row0;
  std::vector<int> item_t0, item_t1, item_slot;  // task range, partial slot (-1: direct)
  int nslot = 0;                                  // partial slots of kFmmRows complex
  std::vector<int> red_out, red_row0, red_slot0, red_g;
  std::vector<int64_t> in_base, sym_base, out_base;
};

// M2L of every tree level and wave as matrix products on the matrix cores.
// Product g (one level li, one wave w, order P, N = 2P + 1 rows):
//   L_b[k] = sum_o sum_j s^o_{j-k} M_{src(b,o)}[j],
// the Toeplitz matrix of offset o (symbol s^o, shared by every box pair at
// that offset) times the gathered source multipoles.  The level's boxes,
// grouped by their position in the parent (the four positions have
// different interaction lists; the top level is one group), form column
// tiles of kM2lCols target boxes; a tile's entries are the offsets any of its
// boxes uses, each with the pool index of s^o_0 and one source box per
// column (-1: none).  A work item (one wavefront) is kM2lRowTiles row tiles of
// 16 rows of one tile over a contiguous group of its entries (the row tiles
// share the multipole operand); with G > 1 groups per tile the items write
// partial slots that a reduction adds in a fixed order.
constexpr int kM2lCols = 16;
constexpr int kM2lRowTiles = 2;
struct M2lPlan {
  // per product g
  std::vector<int> g_li, g_w, g_P, g_G, g_nb;
  std::vector<int64_t> g_off, g_poff;   // expansions of (li, w); partial slots (complex)
  std::vector<double> g_flops;          // 8 (2P+1)^2 per (target, source) pair, per RHS
  std::vector<double> g_symmax;         // largest |s| of the product's symbols
  std::vector<int> g_item0;             // items of g: [g_item0[g], g_item0[g+1])
  // tiles and entries (ids over all products)
  std::vector<int> tile_ptr, tile_box;  // [ntiles+1], [ntiles * kM2lCols]
  std::vector<int64_t> ent_sym;         // [entries] pool index of s_0
  std::vector<int> ent_src;             // [entries * kM2lCols]
  // work items
  std::vector<int> it_g, it_rt, it_tile, it_e0, it_e1, it_slot;
  int64_t part_len = 0;                 // complex elements of the partial slots per RHS
};
struct M2lDev {
  int *g_P = nullptr, *g_G = nullptr, *g_nb = nullptr;
  int64_t *g_off = nullptr, *g_poff = nullptr;
  int *tile_ptr = nullptr, *tile_box = nullptr, *ent_src = nullptr;
  int64_t *ent_sym = nullptr;
  int *it_g = nullptr, *it_rt = nullptr, *it_tile = nullptr, *it_e0 = nullptr, *it_e1 = nullptr,
      *it_slot = nullptr;
};

struct FmmDev {
  int *ptr = nullptr, *in_P = nullptr, *sym_L = nullptr, *sgn = nullptr, *out_P = nullptr;
  int *item_out = nullptr, *item_row0 = nullptr;
  int *item_t0 = nullptr, *item_t1 = nullptr, *item_slot = nullptr;
  int *red_out = nullptr, *red_row0 = nullptr, *red_slot0 = nullptr, *red_g = nullptr;
  int64_t *in_base = nullptr, *sym_base = nullptr, *out_base = nullptr;
};

struct FmmPlan {
  int Lf = 0, Lt = 0;
  double S0 = 0.0;
  std::vector<FmmLevel> levels;  // index 0 = top level Lt
  int64_t exp_len = 0;           // complex elements of all expansions (per RHS)
  int max_slots = 0;             // largest partial-slot count over the launches
  std::vector<int> nbr_ptr, nbr_idx;
  std::vector<int64_t> part_sym;
  std::vector<FmmLaunch> launches;
  M2lPlan m2l;
  std::vector<cd> pool;
  int64_t n_m2l = 0;
};

int fmm_order(double k, double side, int p, double digits);
// compile-time order bucket of the kernels for a largest order pmax
int pm_bucket(int pmax);

}  // namespace ems

// Device buffers and sizes owned by a handle.
struct ems_handle {
  std::string err;
  int device = 0;
  bool have_media = false, have_particles = false, have_s = false, built = false;
  ems::Media md{};
  ems::SommerfeldSpec somm;

  int n = 0, pmax = 0;
  int64_t ncoef = 0;
  std::vector<double> xy, R;
  std::vector<int> p;
  std::vector<int64_t> off;      // [n+1] complex offsets in the ABI layout
  std::vector<ems::cd> S_host;   // ABI order, row-major per particle
  std::vector<int64_t> S_off;    // [n+1]

  // node table
  ems::NodeTable nodes;
  int q = 0;

  // device state
  double *d_xy = nullptr;        // [n][2]
  int *d_p = nullptr;            // [n]
  int64_t *d_off = nullptr;      // [n+1]
  double2 *d_S = nullptr;        // packed S, transposed per particle (column-major)
  float2 *d_S32 = nullptr;       // complex64 copy for the mixed form
  int64_t *d_Soff = nullptr;     // [n+1]
  // node table on device (structure of arrays)
  double2 *d_xi = nullptr, *d_w = nullptr, *d_sp = nullptr, *d_ss = nullptr;
  double2 *d_R = nullptr;        // [q][4]
  double2 *d_dR = nullptr;       // [q][8]: dR/dlambda_b, dR/dmu_b (substrate), row-major 2x2
  double2 *d_Tu = nullptr;       // [q][4]: transmission into the substrate, row-major 2x2
  double2 *d_spb = nullptr, *d_ssb = nullptr;  // [q]: s of the substrate's P and S waves
  double2 *d_Vp = nullptr, *d_Vs = nullptr;  // [q][2 PMb + 1]: (-i zeta)^n, |n| <= pmax, 0 beyond
  double2 *d_Eagg = nullptr, *d_Edis = nullptr;  // tabulated exponentials (optional)
  float2 *d_Eagg32 = nullptr, *d_Edis32 = nullptr;  // complex64 copies for the mixed form (optional)
  // adjoint tables (optional): conj(E_dis) in the aggregate layout, conj(E_agg)
  // in the disaggregate layout, and their power tables conj(V) (-1)^n, conj(V)
  double2 *d_EaggA = nullptr, *d_EdisA = nullptr;
  double2 *d_VpA_agg = nullptr, *d_VsA_agg = nullptr, *d_VpA_dis = nullptr, *d_VsA_dis = nullptr;
  // depth order of the table rows / columns and the per-node and per-particle
  // ranges of the truncated contractions (with the tables)
  int *d_sperm = nullptr, *d_kcut = nullptr, *d_jr = nullptr;
  // register form of the exponentials (every form whose tables were not
  // built): node coefficients [variant][wave][q], particle positions in depth
  // order
  double4 *d_gco = nullptr;
  double2 *d_xys = nullptr;
  bool somm_tab = true;  // tabulate the exponentials at set-up where they fit
  double depth_kept = 1.0, depth_min = 0.0;
  // the same for receivers shallower than every particle (field evaluation)
  int *d_kcut_f = nullptr, *d_jr_f = nullptr;
  double cut_f_depth = -1.0;
  // tile candidate of the matrix-core kernels [aggregate/disaggregate][FP64/FP32]
  // [one / several right-hand sides]; -1: built-in default (ems_autotune sets it)
  int mfma_cfg[2][2][2] = {{{-1, -1}, {-1, -1}}, {{-1, -1}, {-1, -1}}};
  bool p_uniform = false;
  double etab_budget_gb = 96.0;
  // workspaces (sized for ws_nrhs right-hand sides)
  int ws_nrhs = 0;
  int agg_chunks = 0, dis_chunks = 0;
  double2 *d_agg = nullptr;      // [nrhs][2 waves][agg_chunks][q]
  double2 *d_refl = nullptr;     // [nrhs][2][q] reflected amplitudes (weights folded in)
  double2 *d_dis = nullptr;      // [nrhs][dis_chunks][ncoef] partial local coefficients
  double2 *d_free = nullptr;     // [nrhs][ncoef]
  double2 *d_xpad = nullptr;     // [nrhs][2][n][16 NU] aggregate operand (matrix-core form)
  double2 *d_bpad = nullptr;     // [nrhs][2][q][16 NU] disaggregate operand (matrix-core form)
  int64_t n_pairs = 0;
  bool near_fp64 = false;        // mixed form keeps the near field in FP64 (FP32 range)
  bool somm_fp64 = false;        // mixed form keeps the Sommerfeld contractions in FP64
  // algorithmic flops per right-hand side (complex multiply-add = 8)
  double flops_graf = 0.0;   // direct Graf sum over the pairs the kernel visits
  double flops_s = 0.0;      // S multiply, 8 sum (4 p_m + 2)^2

  // free-space FMM
  int fmm_mode = 0;            // 0 auto, 1 direct, 2 FMM
  int fmm_leaf = 6, fmm_top = 64;
  double fmm_digits = 13.0;
  bool fmm_on = false;
  ems::FmmPlan fmm;
  std::vector<ems::FmmDev> fmm_dev;
  ems::M2lDev m2l_dev;
  double2 *d_m2l_part = nullptr;  // [nrhs][m2l.part_len] M2L partial slots
  double2 *d_pool = nullptr, *d_mult = nullptr, *d_loc = nullptr;
  double2 *d_fmm_part = nullptr;  // [nrhs][max_slots][kFmmRows] task-group partials
  double2 *d_nsym = nullptr;      // near-pair symbols [pair][2][4 PMb + 1] (optional)
  int *d_nbr_ptr = nullptr, *d_nbr_idx = nullptr;
  int64_t *d_nbr_off = nullptr;  // per near pair: coefficient offset of the partner
  int *d_nbr_p = nullptr;        // per near pair: order of the partner
  double2 *d_adj1 = nullptr, *d_adj2 = nullptr;  // adjoint free-part scratch
  size_t adj_bytes = 0;

  // kernel timing (ems_profile)
  bool prof = false;
  struct ProfRec {
    const char *name;
    hipEvent_t a, b;
    double flops;  // algorithmic floating-point operations of the launch
  };
  std::vector<ProfRec> prof_recs;

  // GMRES workspace
  double2 *d_V = nullptr;        // Krylov basis
  size_t V_bytes = 0;
  double2 *d_tmp = nullptr;      // scratch vectors
  size_t tmp_bytes = 0;
  double *d_red = nullptr;       // reduction partials
  size_t red_bytes = 0;
  // captured applies (ems_apply_graph): key (x, y, nrhs, flags, adjoint) ->
  // (executable graph, workspace epoch at capture); any reallocation of an
  // apply workspace bumps ws_epoch and forces a new capture
  std::map<std::tuple<const void *, void *, int, int, int>, std::pair<hipGraphExec_t, uint64_t>>
      graphs;
  uint64_t ws_epoch = 0;
  hipStream_t cap_stream = nullptr;  // capture/replay stream for callers on the null stream
  hipEvent_t cap_ev[2] = {nullptr, nullptr};
  // operator with orders p + 1 and S = I on the same geometry (gradient)
  ems_handle *ext = nullptr;
  // mixed-precision refinement: residual and correction [nrhs][ncoef]
  double2 *d_irR = nullptr, *d_irD = nullptr;
  size_t ir_bytes = 0;

  // cluster block-Jacobi preconditioner (built by the first solve or
  // ems_precond_apply after a build): clusters of at most pc_cap unknowns,
  // rows of cluster c = global coefficient indices d_pc_rows[d_pc_rptr[c] ..
  // d_pc_rptr[c+1]), inverse blocks complex64 column-major at d_pc_ioff[c]
  int pc_cap = 512;
  bool pc_built = false;
  int pc_nc = 0, pc_n2 = 0, pc_bmax = 0;
  int *d_pc_rptr = nullptr, *d_pc_rows = nullptr, *d_pc_nb = nullptr;
  int64_t *d_pc_ioff = nullptr;
  float2 *d_pc_inv = nullptr;
  int64_t pc_store = 0;          // complex64 entries of the inverse store
  double pc_setup_s = 0.0;
  double2 *d_pcz = nullptr;      // preconditioned vectors [2][nrhs][ncoef]
  size_t pcz_bytes = 0;
  // estimated relative residual per iteration of the last solve
  std::vector<double> hist;
  int reorth = 0;                // second Gram-Schmidt passes in the last solve
  ems_progress_fn progress = nullptr;
  int progress_every = 0;
  void *progress_user = nullptr;
};

namespace ems {

// threads of the one-workgroup-per-particle kernels: one lane per row of a
// particle block, 2 (2 pmax + 1) rows
inline int part_threads(const ems_handle *h) { return 2 * (2 * h->pmax + 1) <= 64 ? 64 : 128; }

// Records HIP events around one launch when profiling is on.
struct ProfScope {
  ems_handle *h;
  hipStream_t st;
  size_t idx;
  ProfScope(ems_handle *h_, const char *name, hipStream_t s, double flops = 0.0)
      : h(h_), st(s), idx(0) {
    if (!h->prof) return;
    ems_handle::ProfRec r{name, nullptr, nullptr, flops};
    (void)hipEventCreate(&r.a);
    (void)hipEventCreate(&r.b);
    (void)hipEventRecord(r.a, st);
    h->prof_recs.push_back(r);
    idx = h->prof_recs.size();
  }
  ~ProfScope() {
    if (idx) (void)hipEventRecord(h->prof_recs[idx - 1].b, st);
  }
};

// ---- kernel launchers (defined in the .hip files) --------------------------
hipError_t launch_graf_direct(const ems_handle *h, const double2 *x, double2 *out, int nrhs,
                              bool adjoint, bool mixed, hipStream_t st);
int build_fmm(const ems_handle *h, FmmPlan &F, std::string &err);
hipError_t launch_near_symbols(ems_handle *h, const int *pair_tgt, hipStream_t st);
// mixed: the M2L runs on FP32 matrix cores where its symbols fit FP32
hipError_t launch_fmm(const ems_handle *h, const double2 *x, double2 *fre, int nrhs, bool mixed,
                      hipStream_t st);
hipError_t launch_conj_flip(const ems_handle *h, const double2 *in, double2 *out, int nrhs,
                            hipStream_t st);
// cut: the depth truncation's per-node prefixes (aggregate) or per-particle
// node ranges (disaggregate) to use; nullptr = the build's (other end of
// every pair at the shallowest particle's depth).
hipError_t launch_somm_aggregate(const ems_handle *h, const double2 *x, int nrhs, bool adjoint,
                                 bool mixed, hipStream_t st, const int *cut = nullptr);
hipError_t launch_somm_aggregate_mfma(const ems_handle *h, const double2 *x, int nrhs, int prec,
                                      int idx, hipStream_t st, bool adj = false,
                                      const int *cut = nullptr);
hipError_t launch_somm_disaggregate_mfma(const ems_handle *h, int nrhs, int prec, int idx,
                                         hipStream_t st, bool adj = false,
                                         const int *cut = nullptr);
int mfma_candidate(int kernel, int prec, int idx, int *nt, int *rb);
hipError_t launch_somm_reflect(const ems_handle *h, int nrhs, bool adjoint, hipStream_t st,
                               bool transmit = false);
hipError_t launch_etables(ems_handle *h, hipStream_t st);
hipError_t launch_gen_coef(ems_handle *h, hipStream_t st);
// the matrix-core Sommerfeld kernels can run (register form, or tables built)
bool somm_mfma_ready(const ems_handle *h, bool adjoint);
// ... and have an FP32 form for the mixed apply
bool somm_mfma_fp32(const ems_handle *h);
hipError_t launch_somm_disaggregate(const ems_handle *h, int nrhs, bool adjoint, bool mixed,
                                    hipStream_t st, const int *cut = nullptr);
// True when the disaggregate of this apply writes complex64 partial sums (the
// FP32 matrix-core kernel of a forward mixed apply).
bool somm_dis_c64(const ems_handle *h, bool adjoint, bool mixed);
// y = x*idscale - S^{(H)} (a_free + sum of disaggregate partials) per flags;
// mixed: S from its complex64 copy, the partials as somm_dis_c64 says.
hipError_t launch_combine(const ems_handle *h, const double2 *x, double2 *y, int nrhs,
                          int flags, bool adjoint, bool mixed, hipStream_t st);
// plane-wave local coefficients (before S): c [nrhs][ncoef]
hipError_t launch_incident(const ems_handle *h, const int *wave, const double *angle,
                           const double2 *Rinc, int nrhs, double2 *c, hipStream_t st);
hipError_t launch_s_multiply(const ems_handle *h, const double2 *c, double2 *y, int nrhs,
                             hipStream_t st);

// ---- small BLAS-like kernels for GMRES -------------------------------------
// (the basis V in complex128, or complex64 for the mixed inner solves)
// out[i] = conj(V_i) . w   (i < k)
hipError_t launch_mdot(const double2 *V, int64_t ldv, int k, const double2 *w, int64_t n,
                       double2 *out_dev, double *scratch, hipStream_t st);
hipError_t launch_mdot(const float2 *V, int64_t ldv, int k, const double2 *w, int64_t n,
                       double2 *out_dev, double *scratch, hipStream_t st);
// w -= sum_i V_i c_i
hipError_t launch_mupdate(const double2 *V, int64_t ldv, int k, const double2 *c, double2 *w,
                          int64_t n, hipStream_t st);
hipError_t launch_mupdate(const float2 *V, int64_t ldv, int k, const double2 *c, double2 *w,
                          int64_t n, hipStream_t st);
// dst = s src narrowed to complex64; dst = src widened to complex128
hipError_t launch_copy_scaled(const double2 *src, float2 *dst, int64_t n, double s,
                              hipStream_t st);
hipError_t launch_widen(const float2 *src, double2 *dst, int64_t n, hipStream_t st);
hipError_t launch_norm2(const double2 *w, int64_t n, double *out_dev, double *scratch,
                        hipStream_t st);
hipError_t launch_scale(double2 *w, int64_t n, double s, hipStream_t st);
hipError_t launch_copy_scaled(const double2 *src, double2 *dst, int64_t n, double s,
                              hipStream_t st);
// y += sum_i V_i c_i
hipError_t launch_maccum(const double2 *V, int64_t ldv, int k, const double2 *c, double2 *y,
                         int64_t n, hipStream_t st);
hipError_t launch_maccum(const float2 *V, int64_t ldv, int k, const double2 *c, double2 *y,
                         int64_t n, hipStream_t st);
hipError_t launch_axpy(double2 *y, const double2 *x, int64_t n, double a, hipStream_t st);
// Block operations of the block Krylov solver (block.hip), s <= 64 columns:
// H[i][c] = sum_r conj(V_i[r]) W_c[r] (k x s, row-major), with part holding
// bdot_chunks(k, n) k s partial sums; out_c = beta out_c + alpha sum_i V_i H[i][c].
int bdot_chunks(int k, int64_t n);
hipError_t launch_bdot(const double2 *V, int k, const double2 *W, int s, int64_t n, double2 *H,
                       double2 *part, hipStream_t st);
hipError_t launch_baxpy(const double2 *V, int k, const double2 *H, int s, int64_t n,
                        double2 *out, double alpha, double beta, hipStream_t st);

// field evaluation
hipError_t launch_repack(const ems_handle *src, const ems_handle *dst, const double2 *in,
                         double2 *out, int nrhs, hipStream_t st);
hipError_t launch_grad_centres(const ems_handle *h, const ems_handle *e, const double2 *gam,
                               const double2 *mu, const double2 *ae, const double2 *a0e,
                               const double2 *fe, const double2 *ze, int nrhs, double *dxy,
                               hipStream_t st);
hipError_t launch_lame_ig(const ems_handle *h, int nrhs, double2 *Ig, hipStream_t st);
hipError_t launch_lame_lam(const ems_handle *h, int nrhs, double2 *Lam, bool accumulate,
                           hipStream_t st);
hipError_t launch_lame_reduce(const ems_handle *h, int nrhs, const double2 *Ig,
                              const double2 *Lam, double *part, int blocks, hipStream_t st);
hipError_t launch_re_dot(int64_t len, const double2 *a, const double2 *b, double *part,
                         int blocks, hipStream_t st);
hipError_t launch_field_direct(const ems_handle *h, const double2 *gamma, int nrhs, int npts,
                               const double *pts, double2 *u, hipStream_t st);
hipError_t launch_field_direct_adjoint(const ems_handle *h, const double2 *res, int nrhs,
                                       int npts, const double *pts, double2 *g, hipStream_t st);
hipError_t launch_field_refl_adjoint(const ems_handle *h, const double2 *res, int nrhs, int npts,
                                     const double *pts, hipStream_t st);
hipError_t launch_field_trans(const ems_handle *h, int nrhs, int npts, const double *pts,
                              double2 *u, hipStream_t st);
hipError_t launch_field_refl(const ems_handle *h, int nrhs, int npts, const double *pts,
                             double2 *u, hipStream_t st);

// Scattering matrices of non-circular particles by fundamental solutions
// (shapes.hip).  Per-particle device arrays: kind, a, e^{i theta0} as (ct, st),
// source offset delta, p, bc; Soff [n+1] complex offsets of the packed
// row-major output.
struct MfsBatch {
  const Media *md;
  int npts;
  const int *kind, *p, *bc;
  const double *a, *ct, *st, *delta;
  const int64_t *Soff;
};
hipError_t launch_mfs_smatrices(const MfsBatch &b, int i0, int cnt, double2 *W, int64_t mstride,
                                double2 *E, int64_t estride, int *info, double2 *S,
                                hipStream_t st);
// Batched LU with partial pivoting and back substitution of cnt matrices
// [A | B] (n2 rows, n2 + nrhs columns, column-major, stride mstride): B is
// overwritten by A^{-1} B; info[i] = 1 when a pivot of matrix i is zero.
hipError_t launch_lu_solve_batch(double2 *W, int n2, int64_t mstride, int cnt, int nrhs,
                                 int *info, hipStream_t st);

// Cluster block-Jacobi preconditioner (precond.hip).  A batch is the clusters
// c0 .. c0 + cnt - 1; pairs[5 k ..] = {matrix in the batch, m, l, row offset
// of m, column offset of l} for every ordered pair m != l of its clusters.
struct PcBatch {
  int c0 = 0, cnt = 0;
  const int *pairs = nullptr;
  int npairs = 0;
};
hipError_t launch_pc_factor_batch(const ems_handle *h, const PcBatch &bt, double2 *W, int n2,
                                  int64_t mstride, int *info, hipStream_t st);
hipError_t launch_pc_apply(const ems_handle *h, const double2 *x, double2 *y, int nrhs,
                           bool adjoint, hipStream_t st);

}  // namespace ems
