/*
 * ems.h -- C ABI of the MI355X (gfx950) multiple-scattering operator library.
 *
 * Elastic scattering by many rigid or traction-free particles buried in the
 * lower layer of a two-layer medium with a welded flat interface (Zhang, He,
 * Lai, "A fast solver for many-particle elastic scattering in layered media").
 *
 * Frame (Section 2): interface y = 0; the particles and their host medium are
 * in y < 0; the other medium ("substrate") fills y > 0.  Every coefficient
 * vector crossing this ABI is complex128, interleaved (re, im), laid out as
 * [nrhs][sum_m 2(2 p_m + 1)], and per particle [alpha_{-p..p}, beta_{-p..p}]
 * (outgoing coefficients of grad H_n(kp r) e^{i n th} and
 * grad^perp H_n(ks r) e^{i n th}, Section 4.1; truncation Z_p, Section 4.1
 * remark; block order of the multiple-scattering system, Section 4.2).
 *
 * Ownership: the caller owns every buffer passed in; "host" pointers are read
 * (or written) during the call only; "device" pointers must stay valid until
 * the work queued on the given stream has finished.  Calls that take a stream
 * queue work on it and return without waiting, except ems_build and
 * ems_solve, which finish before returning.  A handle must not be used by two
 * threads at once.
 *
 * Errors: 0 = OK, > 0 warning, < 0 error; ems_last_error() returns a message.
 * No C++ exception crosses this boundary.
 */
#ifndef EMS_H
#define EMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EMS_OK 0
#define EMS_NOT_CONVERGED 1       /* solve: iteration limit reached            */
#define EMS_ERR_ARG (-1)          /* bad argument (null, size, range)          */
#define EMS_ERR_GEOMETRY (-2)     /* overlapping disks, disk crossing y = 0    */
#define EMS_ERR_HIP (-3)          /* a HIP runtime call failed                  */
#define EMS_ERR_OOM (-4)          /* device allocation failed                   */
#define EMS_ERR_STATE (-5)        /* call order (e.g. apply before build)       */
#define EMS_ERR_NUMERIC (-6)      /* NaN / Inf in an input, singular 4x4 system */
#define EMS_ERR_UNIMPLEMENTED (-7)

typedef struct ems_handle ems_handle;
typedef void *ems_stream_t; /* a hipStream_t; NULL means the default stream */

/* Lame parameters and density of one homogeneous layer (Section 2; the paper
 * sets rho = 1, the library keeps it: kp = omega sqrt(rho/(lambda+2mu)),
 * ks = omega sqrt(rho/mu)). */
typedef struct {
  double lambda, mu, rho;
} ems_medium;

/* host = the particle layer (y < 0), substrate = y > 0; omega > 0. */
typedef struct {
  ems_medium host, substrate;
  double omega;
} ems_media;

/* Sommerfeld quadrature on the xi axis (Section 5.1).
 *  kind 0: the paper's hyperbolic-tangent contour xi(t) = t - i delta tanh t,
 *          t in [-t_max, t_max], trapezoidal rule with q nodes;
 *  kind 1: real axis; around the branch points (+-kp, +-ks of both layers)
 *          composite Gauss-Legendre panels graded towards each branch point
 *          with a xi = k +- u^2 substitution panel next to it, panel length
 *          from the horizontal extent and depth of the particle cloud; the
 *          tails out to +-t_max by the trapezoidal rule on a smooth (erfc)
 *          partition of unity; q is an output (node count);
 *  kind 2: user nodes: q entries of nodes = [Re xi, Im xi, Re w, Im w];
 *  kind 3: as kind 1 but Gauss-Legendre panels on the tails too.
 * t_max <= 0 asks the library to choose it from the depth of the shallowest
 * particle and the largest p (decay of exp(-|xi| D)(2|xi|/k)^(2p)).
 * panel_scale multiplies the default panel length of kind 1 (1 = default);
 * panel_order is the Gauss-Legendre order of the kind 1 panels (0 = 64);
 * tail_factor scales the trapezoidal density of the kind 1 tails (0 = 1).
 * depth_cut: with the tabulated (matrix-core) contractions, a pair of a real
 * node xi and a particle at depth d is left out of the aggregate and the
 * disaggregate when exp(-Re s(xi) d) (2|xi|/k + 1)^p, times the same factor
 * of the shallowest particle, is below depth_cut times the peak of the
 * t_max bound for the shallowest pair (0 = 1e-26; < 0: every pair kept). */
typedef struct {
  int32_t kind;
  int32_t q;
  double t_max;
  double delta;
  double panel_scale;
  const double *nodes; /* host, kind 2 only */
  int32_t panel_order;
  double tail_factor;
  double depth_cut;
} ems_sommerfeld;

/* Plane wave of unit displacement, |a| < pi/2.
 *  wave 0: P from the particle side towards the interface, direction
 *          d = (sin a, cos a) in the paper frame, d e^{i kp d.x};
 *  wave 1: SV from the particle side, d_perp e^{i ks d.x}, d_perp = (-d2, d1);
 *  wave 2: P sent from the substrate, d = (sin a, -cos a), d e^{i kpb d.x}
 *          (Section 7.3's plane-wave setup: the particles see the wave
 *          transmitted through the interface);
 *  wave 3: SV sent from the substrate, d_perp e^{i ksb d.x}. */
typedef struct {
  int32_t wave;
  double angle;
} ems_plane_wave;

/* Elastic point source in the substrate (Section 3.2): position (x0, y0)
 * with y0 > 0 (paper frame), polarisation (alpha1, alpha2); the incident
 * field is Phi(x, x0) alpha with Phi the substrate's Green's tensor
 * 1/(rho omega^2) (ks^2 g_ks I + grad grad^T (g_ks - g_kp)), g_k = (i/4) H_0(k r). */
typedef struct {
  double x0, y0, alpha1, alpha2;
} ems_point_source;

typedef struct {
  double tol;        /* relative residual target ||b - A x|| / ||b||          */
  int32_t restart;   /* Krylov dimension before a restart (<= 0: as many
                        basis vectors as fit in half of the free device
                        memory, at most 5000)                                  */
  int32_t maxit;     /* total inner iterations                                 */
  int32_t precision; /* 0: FP64 GMRES; 1: FP32 contractions in the inner
                        solve with FP64 iterative refinement                    */
  double inner_tol;  /* precision 1: relative tolerance of each inner solve
                        (<= 0: 1e-3, above the floor the FP32 products leave) */
  int32_t precond;   /* 0: none; 1: cluster block-Jacobi right preconditioner
                        (ems_set_precond), M^{-H} for the adjoint solve         */
  int32_t block;     /* 0: independent GMRES per right-hand side (lock-step);
                        1: block GMRES, one Krylov space for each group of up
                        to 64 right-hand sides (precision 0 only); restart
                        then counts block steps (<= 0: from free memory, at
                        most 8192 basis vectors per group) and maxit block
                        steps per group                                      */
} ems_solver_opts;

typedef struct {
  int32_t iters;       /* inner iterations (all RHS, lock-step: per RHS)      */
  int32_t outer_iters; /* refinement sweeps (precision 1), else 1             */
  int32_t converged;
  double relres;       /* max over RHS of the final FP64 relative residual,
                          computed from b - A x (not the GMRES estimate)      */
  double seconds;      /* wall time of the call, preconditioner set-up included */
  int32_t restart;     /* Krylov dimension used                               */
  double precond_seconds; /* set-up time of the preconditioner (0 if none)    */
  int32_t reorth;      /* Arnoldi steps that needed a second Gram-Schmidt pass */
} ems_solve_info;

typedef struct {
  int32_t n;            /* particles                                          */
  int32_t p_max;
  int64_t n_coeff;      /* complex unknowns per right-hand side               */
  int32_t q;            /* Sommerfeld nodes                                   */
  double t_max;
  int64_t n_pairs;      /* free-space particle pairs evaluated directly       */
  int32_t fmm_levels;   /* 0 = direct sum                                     */
  int64_t fmm_m2l;      /* multipole-to-local translations per apply          */
  double kp, ks, kpb, ksb;
  double somm_kept;     /* fraction of the Sommerfeld contraction work kept by
                           the depth truncation (1 when the vector-ALU
                           kernels run)                                       */
  int32_t mixed_near_fp64; /* 1: the mixed form keeps the direct / near-field
                              Graf sums in FP64 because their Hankel symbols
                              |H_nu(kp d)|, |nu| <= 2 p_max, at the closest
                              pair could exceed 1e30 (FP32 range)             */
  int32_t mixed_somm_fp64; /* 1: the mixed form runs the matrix-core
                              Sommerfeld contractions in FP64 (the node powers
                              (-i zeta)^n, |n| <= p_max, exceed 1e30, or
                              neither complex64 tables nor the register form
                              are available)                                   */
} ems_build_info;

/* Parts of the operator selected by ems_apply's flags. */
#define EMS_PART_FREE 1      /* T_free: Graf translations (Section 4.2)          */
#define EMS_PART_REFL 2      /* T_refl: Sommerfeld reflected part (Section 5)    */
#define EMS_PART_S 4         /* multiply by the particle S-matrices              */
#define EMS_PART_IDENTITY 8  /* y = x - (...); requires EMS_PART_S               */
#define EMS_APPLY_ALL 15
#define EMS_MIXED 256        /* FP32 contractions (FP64 coefficient generation)  */

/* Create an empty handle on the current HIP device. */
int ems_create(ems_handle **out);
void ems_destroy(ems_handle *h);
const char *ems_last_error(const ems_handle *h);

/* Materials and frequency (Section 2).  Host data. */
int ems_set_media(ems_handle *h, const ems_media *m);

/* Particles (Section 2, well-separated enclosing disks, Section 4.3): n centres
 * xy[n][2] in the paper frame, enclosing radii R[n], truncation orders
 * p[n] in [1, 16].  Host data, copied.  Validation at ems_build:
 * |x_m - x_l| > R_m + R_l and y_m + R_m < 0, else EMS_ERR_GEOMETRY. */
int ems_set_particles(ems_handle *h, int32_t n, const double *xy, const double *R,
                      const int32_t *p);

/* Per-particle scattering matrices (Section 4.1 and 4.3), host data, copied:
 * S + 2*offsets[m] doubles hold particle m's (4p_m+2)^2 complex matrix,
 * row-major, rows and columns in the [alpha, beta] / [a, b] order above.
 * offsets has n+1 entries counted in complex elements. */
int ems_set_smatrices(ems_handle *h, const double *S, const int64_t *offsets);

/* Per-particle scattering matrices as turned copies of a few prototypes
 * (Section 4.3: finitely many distinct shapes, placed at any orientation):
 * particle m gets S_m = D S_{which[m]} D^H with D = diag(e^{-i n theta0[m]})
 * over [alpha_{-p..p}, beta_{-p..p}] (the coefficients of a shape turned by
 * theta0 counter-clockwise).  Host data, read during the call: nproto
 * prototypes packed row-major as in ems_set_smatrices, proto_off[nproto+1]
 * complex offsets from 0; which[n] in [0, nproto) and theta0[n] per particle.
 * A prototype's size must be (4 p_m + 2)^2 of every particle that uses it,
 * else EMS_ERR_ARG.  Replaces any matrices set before. */
int ems_set_smatrices_rotated(ems_handle *h, int32_t nproto, const double *S_proto,
                              const int64_t *proto_off, const int32_t *which,
                              const double *theta0);

/* Closed-form scattering matrix of a disk of radius a (Section 4.1: boundary
 * condition imposed mode by mode; bc 0 rigid u = 0, bc 1 traction-free).
 * Writes (4p+2)^2 complex128 row-major into host memory S_out. */
int ems_smatrix_disk(const ems_media *m, double a, int32_t p, int32_t bc, double *S_out);

/* Scattering matrices of non-circular particles (Section 4.3), generated on
 * the GPU for the handle's particles (after ems_set_media and
 * ems_set_particles; orders p from the particles).  Host arrays, one entry
 * per particle: kind 0 circle of radius a, 1 ellipse with semi-axes a and
 * a/2, 2 five-arm star r(t) = a (1 + 0.3 cos 5t), and the paper's family
 * r(t) = a1 + a2 cos(a3 t) of Section 7 with a1 = a, a2 = a/4: 3 pear
 * (a3 = 3), 4 starfish (a3 = 5); each about the particle centre and turned
 * by theta0 (radians, counter-clockwise in the paper frame); bc 0 rigid
 * (u = 0), 1 traction-free.  The shape must lie inside the enclosing radius
 * R (a, a, 1.3 a, 1.25 a, 1.25 a), else EMS_ERR_GEOMETRY.
 * Discretisation (the paper uses a boundary integral equation; here the
 * method of fundamental solutions): npts compressional and npts shear
 * monopoles H_0 at z(t_j + i delta), t_j = 2 pi j / npts, the boundary
 * condition collocated at z(t_j), Graf's addition theorem projects the
 * monopoles onto the outgoing coefficients.  npts a multiple of 8 in
 * [16, 256] (0 = 256); delta <= 0 selects 0.3 / 0.2 / 0.12 / 0.2 / 0.16 by
 * kind.
 * S_out (device): the matrices in the packing ems_set_smatrices reads
 * (row-major (4p_m+2)^2 per particle, particle m at complex offset
 * sum_{l<m} (4p_l+2)^2).  Finishes before returning; allocates and frees
 * its device workspace (about 16 (2 npts)(2 npts + 8 pmax + 4) bytes per
 * particle, in batches of at most 6 GiB and 40 % of the free device memory).
 * EMS_ERR_NUMERIC when a pivot of a collocation system is exactly zero. */
int ems_smatrix_shapes(ems_handle *h, const int32_t *kind, const double *a, const double *theta0,
                       const int32_t *bc, int32_t npts, double delta, void *S_out,
                       ems_stream_t stream);

/* Sommerfeld quadrature choice (Section 5.1); default kind 1 when never set. */
int ems_set_sommerfeld(ems_handle *h, const ems_sommerfeld *s);

/* Host-only: the node table that ems_build would use for this cloud (same
 * rules as ems_set_sommerfeld), without touching the GPU.  xy [n][2] and p[n]
 * host.  On entry *q is the capacity of nodes_out (entries of 6 doubles:
 * Re xi, Im xi, Re w, Im w, bp, d where a node of a branch-point panel has
 * xi = bp + d exactly and bp = 0 marks an ordinary node); on return *q is the
 * node count.  nodes_out may be NULL to query the count.  *t_max receives the
 * tail extent used. */
int ems_sommerfeld_nodes(const ems_media *m, const ems_sommerfeld *s, int32_t n,
                         const double *xy, const int32_t *p, int32_t *q, double *nodes_out,
                         double *t_max);

/* Host-only: the depth truncation ems_build applies to the tabulated
 * Sommerfeld contractions of this cloud (rule: ems_sommerfeld.depth_cut;
 * Section 5.1 places t_max by the same decay bound).  q must be the node
 * count ems_sommerfeld_nodes reports.  Outputs, caller-owned host arrays:
 * perm_out[n] = particle indices by increasing depth; kcut_out[2 q] = for
 * wave w (0 P, 1 S) and node j, entry w q + j: how many particles of that
 * order the node keeps (a prefix); range_out[4 n] = entries 2 (w n + i) and
 * 2 (w n + i) + 1: the node range [lo, hi) holding every node that keeps the
 * i-th particle of that order (lo = hi = 0 when none does); *kept_out
 * (optional) = the kept fraction of (node, particle, wave) triples. */
int ems_sommerfeld_depth_cuts(const ems_media *m, const ems_sommerfeld *s, int32_t n,
                              const double *xy, const int32_t *p, int32_t q, int32_t *perm_out,
                              int32_t *kcut_out, int32_t *range_out, double *kept_out);

/* Host-only: the 2x2 reflection R(xi) of upgoing P / S potentials at the
 * welded interface (Section 3.2, the 4x4 continuity system per Fourier mode,
 * density kept), row-major complex128 into R_out[8]. */
int ems_reflection(const ems_media *m, double xi_re, double xi_im, double *R_out);

/* Free-space part (Section 4.2 gives the Graf translations and names the
 * FMM; the library builds a uniform-quadtree Graf FMM).
 *  mode 0: automatic (FMM when n > 1500), 1: direct sum over all pairs,
 *  2: FMM.  leaf: target particles per leaf box (0 = 6); top_boxes: the
 *  coarsest level kept has at most this many occupied boxes, all of whose
 *  non-adjacent pairs interact directly (0 = 64); digits: accuracy target of
 *  the expansion orders (0 = 13). */
typedef struct {
  int32_t mode;
  int32_t leaf;
  int32_t top_boxes;
  double digits;
} ems_fmm;

int ems_set_fmm(ems_handle *h, const ems_fmm *f);

/* How the Sommerfeld contractions obtain the geometric exponentials
 * E(j, m) = exp(s_w(xi_j) y_m -+ i xi_j x_m) of the aggregate (Section 5.4)
 * and the disaggregate (Section 5.3).  tabulate 1 (the default): ems_build
 * tabulates them, 16 B per (node, particle, wave type) for each contraction,
 * plus complex64 copies for the mixed form and the conjugated tables of the
 * adjoint, each set only when it fits in a 96 GB budget and 60 % of free
 * memory.  Every form without tables (tabulate 0: all of them) has the
 * matrix-core kernels form each exponential in registers from four
 * coefficients per node and the particle's position (256 B per node and 16 B
 * per particle; about a quarter slower than reading the tables at 20000
 * particles, order 15).  Clouds whose phases reach 1e9 rad keep the tables or,
 * without them, the vector-ALU kernels.  Takes effect at the next ems_build;
 * EMS_ERR_ARG for another value. */
int ems_set_exponentials(ems_handle *h, int32_t tabulate);

/* Validate, build the node table and the per-node 2x2 reflection R(xi_j)
 * (the 4x4 interface system of Section 3.2 solved per node), pack the S
 * store, allocate device workspace.  Synchronous. */
int ems_build(ems_handle *h, ems_stream_t stream);
int ems_get_info(const ems_handle *h, ems_build_info *out);

/* Operator apply on device buffers x, y (complex128, [nrhs][n_coeff], may not
 * alias): with flags = EMS_APPLY_ALL,
 *   y_m = x_m - S_m ( (T_free x)_m + (T_refl x)_m )
 * the Schur-complement operator of Section 5.2 (free part: Section 4.2,
 * reflected part: Sections 5.3-5.4).  Fewer part bits give the pieces
 * (e.g. EMS_PART_REFL alone returns the raw reflected local coefficients).
 * EMS_MIXED runs the contractions in FP32. */
int ems_apply(ems_handle *h, const void *x, void *y, int32_t nrhs, int32_t flags,
              ems_stream_t stream);

/* Captured apply: the first call for a given (x, y, nrhs, flags, adjoint)
 * runs the apply (ems_apply or ems_apply_adjoint) and records the same
 * launch sequence into a HIP graph; later calls with the same buffers replay
 * it (one launch, no host work per kernel), reading whatever x holds then.
 * The graph contains kernels only (no memory set or copy nodes).  A
 * reallocated workspace (a larger nrhs elsewhere) or a rebuild makes the
 * next call capture again.  On the null stream the replay runs on an internal
 * non-blocking stream joined by events.  Not for concurrent use of one
 * handle. */
int ems_apply_graph(ems_handle *h, const void *x, void *y, int32_t nrhs, int32_t flags,
                    int32_t adjoint, ems_stream_t stream);

/* Operator apply for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * The same operator as ems_apply (forward only; flags as there, EMS_MIXED
 * included; x, y as there), with its per-call workspace (Sommerfeld aggregate
 * and disaggregate partial sums, reflected amplitudes, free-space output, FMM
 * expansions) in one static device array of 256 MiB per GPU instead of
 * handle-owned allocations; nothing is allocated or freed.  The split-K
 * chunk counts of the Sommerfeld contractions are halved until the workspace
 * fits; when it does not fit with one chunk each, EMS_ERR_ARG (use fewer
 * right-hand sides; one right-hand side of the 20000-particle cloud needs
 * about 204 MB: the FMM's M2L partial slots, the padded operands of the
 * Sommerfeld contractions and the free-space output).  The array is shared by every handle and call on that GPU and
 * keeps the last call's contents; each call clears the part it uses first.
 * Calls that overlap on one GPU (two streams, two threads) race on it and
 * must be serialized by the caller.  EMS_ERR_STATE while kernel profiling
 * (ems_profile) is on.  Results equal ems_apply's up to the order in which
 * partial sums are added. */
int ems_apply_noalloc(ems_handle *h, const void *x, void *y, int32_t nrhs, int32_t flags,
                      ems_stream_t stream);

/* Conjugate-transpose apply (same flags; y = x - T^H S^H x for ALL). */
int ems_apply_adjoint(ems_handle *h, const void *x, void *y, int32_t nrhs, int32_t flags,
                      ems_stream_t stream);

/* Right-hand side S_m (a0^m, b0^m) of the S-preconditioned system (Section
 * 4.2) for nrhs plane waves, into device memory rhs [nrhs][n_coeff]: the
 * local expansions of the background field in the host (Section 7.3,
 * (bplan)): incident + interface-reflected waves for waves 0 and 1, the
 * transmitted waves for waves 2 and 3. */
int ems_incident(ems_handle *h, const ems_plane_wave *waves, int32_t nrhs, void *rhs,
                 ems_stream_t stream);

/* GMRES on the operator (Sections 4.2 and 5.2): x0 = 0, nrhs independent
 * systems advanced in lock-step.  b, x device memory [nrhs][n_coeff].
 * precision 0: every apply in FP64.  precision 1 (mixed): iterative
 * refinement, i.e. an FP64 outer residual b - A x and update x += d, with d
 * from an inner GMRES to inner_tol (default 1e-3) whose applies run the
 * contractions in FP32 (EMS_MIXED); an inner solve also ends when its
 * estimate gains less than 10 % over 200 iterations (the FP32 products put a
 * floor under what it can reach); tol is met on the FP64 residual.
 * precond 1 runs every GMRES (outer and inner) on A M^{-1} with the cluster
 * block-Jacobi preconditioner (ems_set_precond), built on first use.
 * Returns EMS_NOT_CONVERGED when maxit (total inner iterations) is reached,
 * EMS_ERR_ARG for tol <= 0, maxit <= 0 or another precision.  Synchronous. */
int ems_solve(ems_handle *h, const void *b, void *x, int32_t nrhs, const ems_solver_opts *o,
              ems_solve_info *info, ems_stream_t stream);

/* The same solver on the conjugate-transpose operator A^H (the adjoint
 * system of a misfit gradient: A^H lambda = (d u / d gamma)^H r).  Same
 * arguments, options and return codes as ems_solve. */
int ems_solve_adjoint(ems_handle *h, const void *b, void *x, int32_t nrhs,
                      const ems_solver_opts *o, ems_solve_info *info, ems_stream_t stream);

/* Cluster block-Jacobi preconditioner of the solves (precond = 1).  The
 * particles are split into spatial clusters of at most max_unknowns
 * coefficients (recursive halving of the cloud across its wider extent); on
 * each cluster c the free-space block of the multiple-scattering system of
 * Section 4.2, B_c = I - S_c T_cc (identity on the particle blocks, -S_m
 * T^{ml} between the cluster's particles m != l, T^{ml} the Graf
 * translation), is inverted on the GPU once per build and stored in complex64
 * (about 8 max_unknowns bytes per unknown).  GMRES then runs on A M^{-1} with
 * M = diag(B_c) and returns x = M^{-1} u.  max_unknowns in [1, 512]
 * (0 = 512, eight particles of order 15; a particle larger than it forms a
 * cluster of its own); the default is 512.  Takes effect
 * at the next set-up (a rebuild or the first preconditioned call). */
int ems_set_precond(ems_handle *h, int32_t max_unknowns);

/* y = M^{-1} x (adjoint = 0) or M^{-H} x (adjoint = 1) with the cluster
 * block-Jacobi preconditioner above; builds it first when needed (then
 * synchronous).  x, y device [nrhs][n_coeff] complex128, may not alias.
 * clusters, max_rows (host, may be NULL) receive the cluster count and the
 * largest cluster's unknowns; setup_s the set-up time. */
int ems_precond_apply(ems_handle *h, const void *x, void *y, int32_t nrhs, int32_t adjoint,
                      int32_t *clusters, int32_t *max_rows, double *setup_s,
                      ems_stream_t stream);

/* Progress report of the solves: fn(iteration, estimated relative residual,
 * user) is called on the calling thread after every `every`-th inner
 * iteration of ems_solve / ems_solve_adjoint (fn = NULL switches it off).
 * The callback must not call into this handle. */
typedef void (*ems_progress_fn)(int32_t iteration, double relres, void *user);
int ems_set_progress(ems_handle *h, ems_progress_fn fn, int32_t every, void *user);

/* Residual history of the last ems_solve / ems_solve_adjoint on this handle:
 * the estimated relative residual after every inner iteration (largest over
 * the right-hand sides; for precision 1 the inner estimate scaled by the
 * outer residual at the start of its refinement sweep).  Host out[cap];
 * *count receives the number of iterations recorded (entries beyond cap are
 * not written). */
int ems_solve_history(const ems_handle *h, double *out, int32_t cap, int32_t *count);

/* Scattered displacement at npts points (Section 5, coupled
 * representation).  Host points (y < 0, outside every enclosing disk):
 * outgoing particle fields plus the reflected Sommerfeld field; substrate
 * points (y > 0): the particles' field transmitted through the interface
 * (the same aggregate with T(xi) in place of R(xi)).  Points on y = 0 are
 * rejected (EMS_ERR_GEOMETRY).  gamma device [nrhs][n_coeff]; pts device
 * [npts][2] doubles; u device [nrhs][npts][2] complex128. */
int ems_eval_scattered(ems_handle *h, const void *gamma, int32_t nrhs, int32_t npts,
                       const double *pts, void *u, ems_stream_t stream);

/* Right-hand side of the S-preconditioned system for nrhs point sources
 * (Section 3.2; the point-source workload of Section 7): S_m times the local
 * expansions, about every particle, of the source field transmitted into
 * the host, formed by Jacobi-Anger (Section 5.3, (ja)) on a Sommerfeld node
 * rule laid out for the source-to-particle pairs.  rhs device
 * [nrhs][n_coeff].  Errors: EMS_ERR_GEOMETRY (y0 <= 0), EMS_ERR_ARG,
 * EMS_ERR_STATE, EMS_ERR_NUMERIC, EMS_ERR_HIP.  Synchronous. */
int ems_incident_point(ems_handle *h, const ems_point_source *src, int32_t nrhs, void *rhs,
                       ems_stream_t stream);

/* Background displacement of nrhs point sources (no particles) at npts
 * points of either layer: host (y < 0), the transmitted field; substrate
 * (y > 0), the Green's tensor field plus its interface reflection.  pts
 * device [npts][2] (y != 0, not at a source), u device [nrhs][npts][2]
 * complex128.  Synchronous. */
int ems_eval_background_point(ems_handle *h, const ems_point_source *src, int32_t nrhs,
                              int32_t npts, const double *pts, void *u, ems_stream_t stream);

/* Background displacement of nrhs plane waves (no particles; Section 7.3,
 * (bplan)) at npts points of either layer: in the layer the wave is sent
 * from, incident + reflected; in the other layer, transmitted.  pts device
 * [npts][2] (y != 0), u device [nrhs][npts][2] complex128.  The total field
 * is this plus ems_eval_scattered of the solved coefficients. */
int ems_eval_background(ems_handle *h, const ems_plane_wave *waves, int32_t nrhs,
                        int32_t npts, const double *pts, void *u, ems_stream_t stream);

/* Conjugate transpose of ems_eval_scattered: g = F^H res, the right-hand
 * side A^H lambda = F^H res of the adjoint system of a receiver misfit
 * J = 1/2 sum |u - u_obs|^2 (res = u - u_obs).  res device [nrhs][npts][2]
 * complex128, pts device [npts][2], g device [nrhs][n_coeff] (overwritten).
 * Receivers must lie in the host (y < 0) outside every enclosing disk. */
int ems_eval_scattered_adjoint(ems_handle *h, const void *res, int32_t nrhs, int32_t npts,
                               const double *pts, void *g, ems_stream_t stream);

/* Gradient of a receiver misfit J = 1/2 sum_r sum_rcv |u_r(x_rcv) - u_obs|^2
 * with respect to the particle centres and the substrate's Lame parameters
 * (adjoint method; the derivative identities of the translation, plane-wave
 * and interface operators of Sections 4-5 applied to the Schur system).
 * Inputs, all for the same nrhs plane waves `waves` (host array):
 *   gamma  device [nrhs][n_coeff]: solutions of A gamma = b (b from ems_incident),
 *   lam    device [nrhs][n_coeff]: solutions of A^H lam = F^H res
 *          (ems_eval_scattered_adjoint, then ems_solve_adjoint),
 *   pts    device [npts][2], res device [nrhs][npts][2]: u - u_obs.
 * Outputs: dxy device [n][2] (dJ/dx_m, dJ/dy_m), dlame host [2]
 * (dJ/dlambda_b, dJ/dmu_b).  The first call after a build constructs an
 * internal operator with orders p + 1 (so p <= 15 here).  Synchronous.
 * Errors: EMS_ERR_ARG, EMS_ERR_STATE, EMS_ERR_GEOMETRY (receivers),
 * EMS_ERR_UNIMPLEMENTED (p = 16, or waves 2 and 3 from the substrate),
 * EMS_ERR_HIP, EMS_ERR_NUMERIC. */
int ems_param_vjp(ems_handle *h, const ems_plane_wave *waves, int32_t nrhs, const void *gamma,
                  const void *lam, int32_t npts, const double *pts, const void *res, double *dxy,
                  double *dlame, ems_stream_t stream);

/* Tile autotuner of the matrix-core Sommerfeld contractions: times each
 * compiled tile shape (nodes or particles per wave NT, right-hand sides per
 * wave RB) of the aggregate and disaggregate, FP64 and (unless the mixed form
 * keeps them in FP64) FP32, with this handle's exponentials (tables or the
 * register form) at batch size nrhs, the best of four launches each, and
 * keeps the fastest for applies with one (nrhs = 1) or several (nrhs > 1)
 * right-hand sides.  chosen (host, may be NULL) receives
 * {agg FP64 NT, RB, agg FP32 NT, RB, dis FP64 NT, RB, dis FP32 NT, RB}
 * (zeros for forms not tuned; all zeros when the vector-ALU kernels run).
 * Synchronous; results of later applies are unchanged up to rounding order. */
int ems_autotune(ems_handle *h, int32_t nrhs, int32_t *chosen, ems_stream_t stream);

/* Per-kernel timing with HIP events recorded on the launch stream around
 * every kernel the library queues.  ems_profile(h, 1) clears and starts
 * recording, ems_profile(h, 0) stops.  ems_profile_read synchronizes on the
 * recorded events and fills up to cap entries (one per kernel name) with the
 * launch count, total milliseconds and the algorithmic floating-point
 * operations of those launches (a complex multiply-add counts 8; taken from
 * the build's own plan: pair lists, FMM task lists, node count; 0 where no
 * count is defined); *count receives the number of names. */
typedef struct {
  char name[40];
  int32_t launches;
  double total_ms;
  double flops;
} ems_kernel_time;

int ems_profile(ems_handle *h, int32_t enable);
int ems_profile_read(ems_handle *h, ems_kernel_time *out, int32_t cap, int32_t *count);

#ifdef __cplusplus
}
#endif
#endif /* EMS_H */
