// Layered reflected part of the operator on a Sommerfeld node set (Section 5).
//
//   aggregate   (multipole-to-Sommerfeld, Section 5.4 Lemma):
//       I_w(j) = sum_m e^{s_w(j) y_m - i xi_j x_m} sum_n c^m_{w,n} (-i zeta_w(j))^n
//   reflect     (interface, Section 3.2 per node; Schur complement, Section 5.2):
//       [RP; RS]_j = w_j R(xi_j) [I_p / (i pi s_p); I_s / (i pi s_s)]
//   disaggregate (Sommerfeld-to-local, Section 5.3, Jacobi-Anger):
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
// Two implementations of the aggregate and disaggregate:
//  * with the geometry exponentials tabulated at set-up (the default when the
//    tables fit in memory), both are skinny complex matrix products on the
//    matrix cores (FP64 MFMA for the FP64 form, FP32 MFMA on complex64
//    tables for the mixed form);
//  * otherwise, and for the adjoint, vector-ALU kernels form each exponential
//    on the fly: lanes own nodes (aggregate) or particles (disaggregate) and
//    the other index is swept in a wave-uniform loop.
// Partial sums over particle chunks (aggregate) and node chunks
// (disaggregate) are written separately and reduced in a fixed order, so
// results are reproducible run to run.
#include <algorithm>
#include <type_traits>

#include "dev.h"
#include "ems_internal.h"

namespace ems {

int pm_bucket(int pmax);

// Vector-ALU forms with the exponentials formed on the fly (used when the
// tables do not fit, and for the adjoint).  MODE 1: forward, 2: adjoint.
template <int PM, bool UNI, int MODE>
__global__ __launch_bounds__(256) void somm_aggregate_kernel(
    int n, int q, int pmax, const double *__restrict__ xy, const int *__restrict__ p,
    const int64_t *__restrict__ off, const double2 *__restrict__ x, int64_t ldx,
    const double2 *__restrict__ xi_t, const double2 *__restrict__ sp_t,
    const double2 *__restrict__ ss_t, const double2 *__restrict__ Vp_t,
    const double2 *__restrict__ Vs_t, double2 *__restrict__ agg, int chunks, int per_chunk,
    int adjoint_unused) {
  constexpr int NM = 2 * PM + 1;
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
  // acc_n = sum_m E(j, m) c^m_n, then I = sum_n V[j][n] acc_n: the 2p+1
  // accumulators are independent chains (same flop count as contracting the
  // modes first).
  double2 acc[NM];
#pragma unroll
  for (int k = 0; k < NM; ++k) acc[k] = make_double2(0.0, 0.0);
  const int m0 = c * per_chunk;
  const int m1 = min(n, m0 + per_chunk);
  const double2 *xr = x + (int64_t)r * ldx;
  auto step = [&](int m, double2 E) {
    const int pm = UNI ? PM : p[m];
    const double2 *cm =
        xr + (UNI ? (int64_t)m * 2 * (2 * PM + 1) : off[m]) + wave * (2 * pm + 1) + pm;
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      const int nn = k - PM;
      if (UNI || (nn >= -pm && nn <= pm)) cfma(acc[k], E, cm[nn]);
    }
  };
  auto expo = [&](int m) {
    const double xm = xy[2 * m], ym = xy[2 * m + 1];
    return cexp(make_double2(a.x * ym + bb.x * xm, a.y * ym + bb.y * xm));
  };
  for (int m = m0; m < m1; ++m) step(m, expo(m));
  // the power table is read only now, so it holds no registers in the loop
  double2 res = make_double2(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    const int nn = k - PM;
    double2 t = Vt[(int64_t)jj * ld + k];
    if (adjoint) {
      t = cconj(t);
      if (nn & 1) t = cscale(t, -1.0);
    }
    cfma(res, t, acc[k]);
  }
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
    int per_chunk, int adjoint_unused) {
  constexpr int NM = 2 * PM + 1;
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
  auto expo = [&](int j) {
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
    return cexp(make_double2(a.x * yl + bb.x * xl, a.y * yl + bb.y * xl));
  };
  auto step = [&](int j, double2 E) {
    const double2 F = cmul(E, gr[j]);
    const double2 *Vj = Vt + (int64_t)j * ld;
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      double2 u = Vj[k];
      if (adjoint) u = cconj(u);
      cfma(acc[k], F, u);
    }
  };
  for (int j = j0; j < j1; ++j) step(j, expo(j));
  if (l < n) {
    double2 *o = dis + ((int64_t)r * chunks + c) * ncoef + off[l] + wave * (2 * pl + 1) + pl;
#pragma unroll
    for (int k = 0; k < NM; ++k) {
      const int nn = k - PM;
      if (nn >= -pl && nn <= pl) o[nn] = acc[k];
    }
  }
}


// ---------------------------------------------------------------------------
// Matrix-core form of the tabulated forward contractions.
//
// Aggregate: for one wave type and one chunk of particles,
//   A[j][k] = sum_m E(j, m) c^m_{k-PM}        (nodes x modes, contracted over m)
//   I_j     = sum_k V[j][k] A[j][k],
// Disaggregate: for one wave type and one chunk of nodes,
//   a^l_{k-PM} = sum_j E(j, l) (RW_j V[j][k])  (particles x modes, contracted over j).
// Both are skinny complex products.  Their long operand, the exponential
// E(j, m), is either read from a table built at set-up (16 B per (node,
// particle), streamed from HBM once per contraction) or, with GEN, formed in
// registers from the particle's position and four per-node coefficients,
//   E = exp((g.x y + g.y x) + i (g.z y + g.w x)),
// (one exp and one sincos per entry on the vector ALU, beside the MFMAs:
// no table, no HBM stream).  The four sign patterns of g give the forward
// and adjoint factors of both contractions (gen_coef_kernel).  A wave
// owns 16*NT rows x 16*NU modes; each step contracts 4 indices (lane group
// kq = lane / 16 supplies index base + kq) with 16x16x4 MFMAs, a complex
// product being three or four real ones (mfma_cstep).  The operands of a
// step are fetched a few steps before its products (SommForm).
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  using Acc = mf_d4;
  using C = double2;
  __device__ static Acc op(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output row held in accumulator element v by lane group kq (column = lane % 16)
  __device__ static int row(int kq, int v) { return kq + 4 * v; }
};
template <> struct Mfma<float> {
  using Acc = mf_f4;
  using C = float2;
  __device__ static Acc op(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int kq, int v) { return 4 * kq + v; }
};

// Per kernel and precision: the complex product form (three or four real
// MFMAs per complex tile) and the operand slots in flight per wave.  Both
// contractions take the 3M form.  Tiles of one right-hand side and at most
// 32 rows are compiled for four wavefronts per SIMD (amdgpu_waves_per_eu),
// which puts the accumulators in ordinary vector registers next to the
// operand slots (at most a few spilled registers), except FP64 tiles of 32
// rows, which take three (the 32-node FP64 aggregate re-reads half the
// coefficient operand of the 16-node one: 2.0 -> 1.92 ms at 20000 particles);
// larger and batched tiles take two, where the candidates below fit without
// spills.
// Measured at 20000 particles, order 15: the FP64 aggregate went from 2.54 to
// 1.92 ms and the FP64 disaggregate from 2.52 (four MFMAs, one slot, three
// waves) to 2.27 ms with 32 particles per wave and 2.16 ms with 16 particles
// and three slots; the FP32 forms to 1.12 and 1.21 ms.  A third FP64
// aggregate slot did not pay.
template <typename T> struct SommForm {
  static constexpr bool kFp32 = std::is_same<T, float>::value;
  static constexpr bool k3MAgg = true, k3MDis = true;
  static constexpr int kSlotsAgg = kFp32 ? 4 : 2;
  // FP64 disaggregate: one slot beside the accumulators of 32 particles,
  // three beside those of 16 particles and one right-hand side when the
  // exponentials come from the table (the register form needs the room)
  static constexpr int slots_dis(int nt, int rb, bool gen) {
    return kFp32 ? 4 : (nt == 1 && rb == 1 && !gen ? 3 : 1);
  }
};

// One step of the complex product.  The 3M form (three real MFMAs):
//   K1 += (Ar + Ai) Br,  K2 += Ar (Bi - Br),  K3 += Ai (Br + Bi),
// with Re = K1 - K3 and Im = K1 + K2 formed once after the loop (the operand
// sums cost three vector adds per lane and step; each accumulator is updated
// once per step, so dependent MFMAs sit 3 NT NC issues apart).  The 4M form
// accumulates Re and Im in k1, k2 directly (k3 unused): first the products
// of every accumulator, then the second ones, so a dependent pair of MFMAs
// sits 2 NT NC issues apart.
template <typename T, int NT, int NC, bool G3>
__device__ __forceinline__ void mfma_cstep(typename Mfma<T>::Acc (&k1)[NT][NC],
                                           typename Mfma<T>::Acc (&k2)[NT][NC],
                                           typename Mfma<T>::Acc (&k3)[NT][NC],
                                           const T (&er)[NT], const T (&ei)[NT], const T (&br)[NC],
                                           const T (&bi)[NC]) {
  if constexpr (!G3) {
#pragma unroll
    for (int u = 0; u < NC; ++u)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        k1[t][u] = Mfma<T>::op(er[t], br[u], k1[t][u]);
        k2[t][u] = Mfma<T>::op(er[t], bi[u], k2[t][u]);
      }
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const T nb = -bi[u];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        k1[t][u] = Mfma<T>::op(ei[t], nb, k1[t][u]);
        k2[t][u] = Mfma<T>::op(ei[t], br[u], k2[t][u]);
      }
    }
    return;
  }
  T es[NT], bd[NC], bs[NC];
#pragma unroll
  for (int t = 0; t < NT; ++t) es[t] = er[t] + ei[t];
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    bd[u] = bi[u] - br[u];
    bs[u] = br[u] + bi[u];
  }
#pragma unroll
  for (int u = 0; u < NC; ++u)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      k1[t][u] = Mfma<T>::op(es[t], br[u], k1[t][u]);
      k2[t][u] = Mfma<T>::op(er[t], bd[u], k2[t][u]);
      k3[t][u] = Mfma<T>::op(ei[t], bs[u], k3[t][u]);
    }
}

// Real and imaginary parts of the 3M accumulators, in place: (K1, K2, K3)
// becomes (Re, Im, -); nothing to do in the 4M form.
template <typename T, int NT, int NC, bool G3>
__device__ __forceinline__ void mfma_cfinish(typename Mfma<T>::Acc (&k1)[NT][NC],
                                             typename Mfma<T>::Acc (&k2)[NT][NC],
                                             const typename Mfma<T>::Acc (&k3)[NT][NC]) {
  if constexpr (!G3) return;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      k2[t][u] = k1[t][u] + k2[t][u];
      k1[t][u] = k1[t][u] - k3[t][u];
    }
}

// Table entries are read exactly once per contraction: non-temporal loads
// keep them from displacing the reused operands (the padded coefficients and
// node operands) in the L2 cache.
typedef double somm_d2v __attribute__((ext_vector_type(2)));
typedef float somm_f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 stream_load(const double2 *p) {
  const somm_d2v v = __builtin_nontemporal_load(reinterpret_cast<const somm_d2v *>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 stream_load(const float2 *p) {
  const somm_f2v v = __builtin_nontemporal_load(reinterpret_cast<const somm_f2v *>(p));
  return make_float2(v.x, v.y);
}

// e^a (cos b, sin b) without the library's large-argument branches, which
// cost registers the matrix-core loops need.  Cody-Waite reduction with
// two-part constants and fused multiply-adds, a = k ln2 + r (|r| <= ln2/2)
// and b = n pi/2 + t (|t| <= pi/4), then Taylor polynomials of the reduced
// arguments: FP64 to degree 13 (e^r, truncation < 5e-18), 15 (sin, < 4e-17)
// and 16 (cos, < 3e-18); the FP32 form (for the complex64 operands of the
// mixed apply) reduces in FP64 and evaluates degree 7, 9 and 10 in FP32
// (truncation < 6e-9).  Valid for |b| < 2^30, which the build checks
// (ems_build keeps the tables or the vector-ALU kernels beyond it); e^a
// flushes to zero below a = -745 (FP64) and -104 (FP32).
constexpr double kLog2e = 1.4426950408889634;       // 1 / ln 2
constexpr double kLn2Hi = 0.6931471805599453;       // ln 2 rounded
constexpr double kLn2Lo = 2.3190468138462996e-17;   // ln 2 - kLn2Hi
constexpr double kTwoOverPi = 0.6366197723675814;   // 2 / pi
constexpr double kPio2Hi = 1.5707963267948966;      // pi / 2 rounded
constexpr double kPio2Lo = 6.123233995736766e-17;   // pi / 2 - kPio2Hi

__device__ __forceinline__ void cexp_reg(double a, double b, double &er, double &ei) {
  const double k = fmin(fmax(__builtin_rint(a * kLog2e), -1100.0), 1100.0);
  double r = fma(-k, kLn2Hi, a);
  r = fma(-k, kLn2Lo, r);
  double p = 1.0 / 6227020800.0;
  p = fma(p, r, 1.0 / 479001600.0);
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  const double e = a < -745.2 ? 0.0 : ldexp(p, (int)k);
  const double n = __builtin_rint(b * kTwoOverPi);
  double t = fma(-n, kPio2Hi, b);
  t = fma(-n, kPio2Lo, t);
  const double z = t * t;
  double sp = -1.0 / 1307674368000.0;
  sp = fma(sp, z, 1.0 / 6227020800.0);
  sp = fma(sp, z, -1.0 / 39916800.0);
  sp = fma(sp, z, 1.0 / 362880.0);
  sp = fma(sp, z, -1.0 / 5040.0);
  sp = fma(sp, z, 1.0 / 120.0);
  sp = fma(sp, z, -1.0 / 6.0);
  const double sn = fma(sp * z, t, t);
  double cp = 1.0 / 20922789888000.0;
  cp = fma(cp, z, -1.0 / 87178291200.0);
  cp = fma(cp, z, 1.0 / 479001600.0);
  cp = fma(cp, z, -1.0 / 3628800.0);
  cp = fma(cp, z, 1.0 / 40320.0);
  cp = fma(cp, z, -1.0 / 720.0);
  cp = fma(cp, z, 1.0 / 24.0);
  cp = fma(cp, z, -0.5);
  const double cs = fma(cp, z, 1.0);
  // quadrant n mod 4: (cos, sin) of b = (cs, sn), (-sn, cs), (-cs, -sn), (sn, -cs)
  const int qd = (int)n & 3;
  const double c0 = (qd & 1) ? sn : cs, s0 = (qd & 1) ? cs : sn;
  er = e * (((qd + 1) & 2) ? -c0 : c0);
  ei = e * ((qd & 2) ? -s0 : s0);
}

__device__ __forceinline__ void cexp_reg(double a, double b, float &er, float &ei) {
  const double k = fmin(fmax(__builtin_rint(a * kLog2e), -200.0), 200.0);
  double r = fma(-k, kLn2Hi, a);
  r = fma(-k, kLn2Lo, r);
  const float rf = (float)r;
  float p = 1.0f / 5040.0f;
  p = fmaf(p, rf, 1.0f / 720.0f);
  p = fmaf(p, rf, 1.0f / 120.0f);
  p = fmaf(p, rf, 1.0f / 24.0f);
  p = fmaf(p, rf, 1.0f / 6.0f);
  p = fmaf(p, rf, 0.5f);
  p = fmaf(p, rf, 1.0f);
  p = fmaf(p, rf, 1.0f);
  const float e = a < -104.0 ? 0.0f : ldexpf(p, (int)k);
  const double n = __builtin_rint(b * kTwoOverPi);
  double t = fma(-n, kPio2Hi, b);
  t = fma(-n, kPio2Lo, t);
  const float tf = (float)t, z = tf * tf;
  float sp = 1.0f / 362880.0f;
  sp = fmaf(sp, z, -1.0f / 5040.0f);
  sp = fmaf(sp, z, 1.0f / 120.0f);
  sp = fmaf(sp, z, -1.0f / 6.0f);
  const float sn = fmaf(sp * z, tf, tf);
  float cp = -1.0f / 3628800.0f;
  cp = fmaf(cp, z, 1.0f / 40320.0f);
  cp = fmaf(cp, z, -1.0f / 720.0f);
  cp = fmaf(cp, z, 1.0f / 24.0f);
  cp = fmaf(cp, z, -0.5f);
  const float cs = fmaf(cp, z, 1.0f);
  const int qd = (int)n & 3;
  const float c0 = (qd & 1) ? sn : cs, s0 = (qd & 1) ? cs : sn;
  er = e * (((qd + 1) & 2) ? -c0 : c0);
  ei = e * ((qd & 2) ? -s0 : s0);
}

// E = exp((g.x y + g.y x) + i (g.z y + g.w x)) at position ps = (x, y).
template <typename T>
__device__ __forceinline__ void gen_exp(const double4 &g, const double2 &ps, T &er, T &ei) {
  cexp_reg(fma(g.x, ps.y, g.y * ps.x), fma(g.z, ps.y, g.w * ps.x), er, ei);
}

// Column tiles: NU tiles of 16 modes for each of RB right-hand sides (tile
// c = k NU + u is right-hand side r0 + k, modes 16 u .. 16 u + 15).  nm =
// 2 PM + 1 of the power tables (PM their padded order), nrhs bounds r0 + k.
// xp: the coefficients in depth order, modes -PM .. 16 NU - 1 - PM
// (somm_xpad_kernel), [nrhs][wave][n][16 NU].
template <typename T, int NU, int NT, int RB, bool GEN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RB > 1 || NT > 2 ? 2 : (NT == 2 && sizeof(T) == 8 ? 3 : 4)))) void somm_aggregate_mfma_kernel(
    int n, int q, int nm, int nrhs, const typename Mfma<T>::C *__restrict__ xp,
    const double2 *__restrict__ Vp_t, const double2 *__restrict__ Vs_t,
    double2 *__restrict__ agg, int chunks, int per_chunk,
    const typename Mfma<T>::C *__restrict__ Etab, const int *__restrict__ kcut,
    const double4 *__restrict__ gco, const double2 *__restrict__ xys) {
  using Acc = typename Mfma<T>::Acc;
  using C = typename Mfma<T>::C;
  constexpr int NC = NU * RB;
  const int lane = threadIdx.x & 63, kq = lane >> 4, i16 = lane & 15;
  const int jb = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 * NT;
  const int c = blockIdx.y, wave = blockIdx.z & 1, r0 = (blockIdx.z >> 1) * RB;
  const C *Ew = Etab + (int64_t)wave * n * q;
  Acc ar[NT][NC], ai[NT][NC], a3[NT][NC];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int u = 0; u < NC; ++u) ar[t][u] = ai[t][u] = a3[t][u] = Acc{0, 0, 0, 0};
  int jl[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) jl[t] = min(jb + 16 * t + i16, q - 1);
  // GEN: the coefficients of the lane's nodes stay in registers
  double4 gc[NT];
  if constexpr (GEN) {
#pragma unroll
    for (int t = 0; t < NT; ++t) gc[t] = gco[(int64_t)wave * q + jl[t]];
  }
  // table rows run through the particles by depth; the wave's nodes keep the
  // first kc of them (the largest count over its nodes)
  int kc = 0;
#pragma unroll
  for (int t = 0; t < NT; ++t) kc = max(kc, kcut[wave * q + jl[t]]);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) kc = max(kc, __shfl_xor(kc, o));
  const int m0 = c * per_chunk, m1 = min(min(n, m0 + per_chunk), kc);
  // A ring of S operand slots, each refilled right after it is consumed:
  // the loads of a step are issued S steps ahead of its products (GEN: a
  // slot holds the particle position instead of table entries).
  constexpr int S = SommForm<T>::kSlotsAgg;
  constexpr int NW = 16 * NU;
  C en[S][NT];
  double2 ps[S];
  C xn[S][NC];
  auto fetch = [&](int sl, int m) {
    const int mc = min(m + kq, m1 - 1);
    if constexpr (GEN) {
      ps[sl] = xys[mc];
    } else {
#pragma unroll
      for (int t = 0; t < NT; ++t) en[sl][t] = stream_load(Ew + (int64_t)mc * q + jl[t]);
    }
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const C *xr = xp + ((int64_t)(min(r0 + k, nrhs - 1) * 2 + wave) * n + mc) * NW + i16;
#pragma unroll
      for (int u = 0; u < NU; ++u) xn[sl][k * NU + u] = xr[16 * u];
    }
  };
  if (m0 < m1) {
#pragma unroll
    for (int sl = 0; sl < S; ++sl) fetch(sl, m0 + 4 * sl);
  }
  for (int m = m0; m < m1; m += 4 * S) {
#pragma unroll
    for (int sl = 0; sl < S; ++sl) {
      const int ms = m + 4 * sl;
      if (sl > 0 && ms >= m1) break;  // uniform over the wave
      const bool ok = ms + kq < m1;
      T er[NT], ei[NT], br[NC], bi[NC];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if constexpr (GEN) {
          gen_exp<T>(gc[t], ps[sl], er[t], ei[t]);
        } else {
          er[t] = en[sl][t].x;
          ei[t] = en[sl][t].y;
        }
      }
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        br[u] = ok ? (T)xn[sl][u].x : T(0);
        bi[u] = ok ? (T)xn[sl][u].y : T(0);
      }
      fetch(sl, ms + 4 * S);
      mfma_cstep<T, NT, NC, SommForm<T>::k3MAgg>(ar, ai, a3, er, ei, br, bi);
    }
  }
  mfma_cfinish<T, NT, NC, SommForm<T>::k3MAgg>(ar, ai, a3);
  // I_j = sum_k V[j][k] A[j][k]; the 16 lanes of a group hold the 16 columns
  const double2 *Vt = wave ? Vs_t : Vp_t;
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    const int r = r0 + k;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = jb + 16 * t + Mfma<T>::row(kq, v);
        const int jc = min(j, q - 1);
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int kk = 16 * u + i16;
          if (kk < nm) {
            const double2 w = Vt[(int64_t)jc * nm + kk];
            const double a = (double)ar[t][k * NU + u][v], b = (double)ai[t][k * NU + u][v];
            re += w.x * a - w.y * b;
            im += w.x * b + w.y * a;
          }
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
          re += __shfl_xor(re, o);
          im += __shfl_xor(im, o);
        }
        if (i16 == 0 && j < q && r < nrhs)
          agg[((int64_t)(r * 2 + wave) * chunks + c) * q + j] = make_double2(re, im);
      }
    }
  }
}

template <typename T, int NU, int NT, int RB, bool GEN>
// bp: the B operand RW_j V[j][k], zero-padded to 16 NU modes
// (somm_bpad_kernel), [nrhs][wave][q][16 NU].
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RB > 1 || NT > 2 ? 2 : (NT == 2 && sizeof(T) == 8 ? 3 : 4)))) void somm_disaggregate_mfma_kernel(
    int n, int q, int nm, int nrhs, const int *__restrict__ p, const int64_t *__restrict__ off,
    const typename Mfma<T>::C *__restrict__ bp, typename Mfma<T>::C *__restrict__ dis,
    int64_t ncoef, int chunks,
    int per_chunk, const typename Mfma<T>::C *__restrict__ Etab, const int *__restrict__ sperm,
    const int2 *__restrict__ jr, const double4 *__restrict__ gco,
    const double2 *__restrict__ xys) {
  using Acc = typename Mfma<T>::Acc;
  using C = typename Mfma<T>::C;
  constexpr int NC = NU * RB, NW = 16 * NU;
  const int PM = nm >> 1;
  const int lane = threadIdx.x & 63, kq = lane >> 4, i16 = lane & 15;
  const int lb = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 * NT;
  const int c = blockIdx.y, wave = blockIdx.z & 1, r0 = (blockIdx.z >> 1) * RB;
  const C *Ew = Etab + (int64_t)wave * q * n;
  Acc ar[NT][NC], ai[NT][NC], a3[NT][NC];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int u = 0; u < NC; ++u) ar[t][u] = ai[t][u] = a3[t][u] = Acc{0, 0, 0, 0};
  int lc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) lc[t] = min(lb + 16 * t + i16, n - 1);
  // GEN: the positions of the lane's particles stay in registers
  double2 pl[NT];
  if constexpr (GEN) {
#pragma unroll
    for (int t = 0; t < NT; ++t) pl[t] = xys[lc[t]];
  }
  // table columns run through the particles by depth; the wave's particles
  // need the hull of their node ranges (empty ranges add nothing)
  int lo = q, hi = 0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int2 r = jr[wave * n + lc[t]];
    if (r.y > r.x) {
      lo = min(lo, r.x);
      hi = max(hi, r.y);
    }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    lo = min(lo, __shfl_xor(lo, o));
    hi = max(hi, __shfl_xor(hi, o));
  }
  const int j0 = max(c * per_chunk, lo), j1 = min(min(q, c * per_chunk + per_chunk), hi);
  // ring of S operand slots, loads issued S steps ahead
  constexpr int S = SommForm<T>::slots_dis(NT, RB, GEN);
  C en[S][NT];
  double4 gj[S];  // GEN: the coefficients of the step's node
  C bn[S][NC];
  auto fetch = [&](int sl, int j) {
    const int jc = min(j + kq, j1 - 1);
    if constexpr (GEN) {
      gj[sl] = gco[(int64_t)wave * q + jc];
    } else {
#pragma unroll
      for (int t = 0; t < NT; ++t) en[sl][t] = stream_load(Ew + (int64_t)jc * n + lc[t]);
    }
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const C *br = bp + ((int64_t)(min(r0 + k, nrhs - 1) * 2 + wave) * q + jc) * NW + i16;
#pragma unroll
      for (int u = 0; u < NU; ++u) bn[sl][k * NU + u] = br[16 * u];
    }
  };
  if (j0 < j1) {
#pragma unroll
    for (int sl = 0; sl < S; ++sl) fetch(sl, j0 + 4 * sl);
  }
  for (int j = j0; j < j1; j += 4 * S) {
#pragma unroll
    for (int sl = 0; sl < S; ++sl) {
      const int js = j + 4 * sl;
      if (sl > 0 && js >= j1) break;  // uniform over the wave
      const bool ok = js + kq < j1;
      T er[NT], ei[NT], br[NC], bi[NC];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if constexpr (GEN) {
          gen_exp<T>(gj[sl], pl[t], er[t], ei[t]);
        } else {
          er[t] = en[sl][t].x;
          ei[t] = en[sl][t].y;
        }
      }
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        br[u] = ok ? (T)bn[sl][u].x : T(0);
        bi[u] = ok ? (T)bn[sl][u].y : T(0);
      }
      fetch(sl, js + 4 * S);
      mfma_cstep<T, NT, NC, SommForm<T>::k3MDis>(ar, ai, a3, er, ei, br, bi);
    }
  }
  mfma_cfinish<T, NT, NC, SommForm<T>::k3MDis>(ar, ai, a3);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int l = lb + 16 * t + Mfma<T>::row(kq, v);
      if (l >= n) continue;
      const int lo_ = sperm[l];
      const int pl = p[lo_];
#pragma unroll
      for (int k = 0; k < RB; ++k) {
        if (r0 + k >= nrhs) break;
        C *o = dis + ((int64_t)(r0 + k) * chunks + c) * ncoef + off[lo_] + wave * (2 * pl + 1) + pl;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int nn = 16 * u + i16 - PM;
          if (nn >= -pl && nn <= pl) {
            C ov;
            ov.x = ar[t][k * NU + u][v];
            ov.y = ai[t][k * NU + u][v];
            o[nn] = ov;
          }
        }
      }
    }
  }
}

#define EMS_AGG_LAUNCH(PMV, UNIV, TABV)                                                    \
  hipLaunchKernelGGL((somm_aggregate_kernel<PMV, UNIV, TABV>), grid, dim3(256), 0, st, h->n,  \
                     h->q, h->pmax, h->d_xy, h->d_p, h->d_off, x, h->ncoef, h->d_xi, h->d_sp,  \
                     h->d_ss, h->d_Vp, h->d_Vs, h->d_agg, h->agg_chunks, per, adjoint ? 1 : 0)
#define EMS_AGG_CASE(PMV)                                                                  \
  case PMV:                                                                                \
    if (mode == 1 && uni) EMS_AGG_LAUNCH(PMV, true, 1);                                    \
    else if (mode == 1) EMS_AGG_LAUNCH(PMV, false, 1);                                     \
    else EMS_AGG_LAUNCH(PMV, false, 2);                                                    \
    break;

// Candidate tile shapes (node or particle tiles NT, right-hand sides per
// wave RB) of the matrix-core kernels, indexed by MfmaCfg::idx; the
// autotuner times them on the handle's own tables.  64 right-hand sides at
// 20000 particles (orders 9-14): FP64 3.29 -> 3.73 and mixed 4.73 -> 5.36
// block applies/s once the batched shapes stopped spilling.
static constexpr int kCand[2][2][4][2] = {
    // [kernel: 0 aggregate, 1 disaggregate][precision: 0 FP64, 1 FP32][candidate] = {NT, RB}
    {{{1, 1}, {1, 2}, {2, 2}, {2, 1}}, {{2, 1}, {4, 1}, {2, 2}, {1, 4}}},
    {{{2, 1}, {1, 1}, {2, 2}, {1, 4}}, {{2, 1}, {4, 1}, {2, 2}, {1, 4}}}};

int mfma_candidate(int kernel, int prec, int idx, int *nt, int *rb) {
  if (kernel < 0 || kernel > 1 || prec < 0 || prec > 1 || idx < 0 || idx > 3) return -1;
  *nt = kCand[kernel][prec][idx][0];
  *rb = kCand[kernel][prec][idx][1];
  return 0;
}

// The aggregate's coefficient operand: x in depth order, one row of 16 NU
// modes per (right-hand side, wave type, particle), zero outside |n| <= p_m,
// so the matrix-core loop reads it without index or order lookups.  The FP32
// contraction takes it in complex64 (it rounds the operand to FP32 anyway),
// which halves the bytes of the operand its waves re-read.
template <typename OC>
__global__ void somm_xpad_kernel(int n, int pmb, int nw, const int *__restrict__ p,
                                 const int64_t *__restrict__ off, const double2 *__restrict__ x,
                                 int64_t ldx, const int *__restrict__ sperm,
                                 OC *__restrict__ xp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int w = blockIdx.y, r = blockIdx.z;
  if (i >= (int64_t)n * nw) return;
  const int m = (int)(i / nw), k = (int)(i - (int64_t)m * nw);
  const int mo = sperm[m], pm = p[mo], nn = k - pmb;
  const double2 v = (nn >= -pm && nn <= pm)
                        ? x[(int64_t)r * ldx + off[mo] + w * (2 * pm + 1) + pm + nn]
                        : make_double2(0.0, 0.0);
  OC o;
  o.x = v.x;
  o.y = v.y;
  xp[((int64_t)(r * 2 + w) * n + m) * nw + k] = o;
}

// The disaggregate's B operand: the reflected node amplitudes times the
// power table, B[r][w][j][k] = g[r][w][j] V_w[j][k], zero beyond the table's
// 2 PM + 1 modes, so the matrix-core loop reads it as one padded row
// (complex64 for the FP32 contraction).
template <typename OC>
__global__ void somm_bpad_kernel(int q, int nm, int nw, const double2 *__restrict__ g,
                                 const double2 *__restrict__ Vp_t,
                                 const double2 *__restrict__ Vs_t, OC *__restrict__ bp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int w = blockIdx.y, r = blockIdx.z;
  if (i >= (int64_t)q * nw) return;
  const int j = (int)(i / nw), k = (int)(i - (int64_t)j * nw);
  const double2 *Vt = w ? Vs_t : Vp_t;
  const double2 v = k < nm ? cmul(g[(int64_t)(r * 2 + w) * q + j], Vt[(int64_t)j * nm + k])
                           : make_double2(0.0, 0.0);
  OC o;
  o.x = v.x;
  o.y = v.y;
  bp[((int64_t)(r * 2 + w) * q + j) * nw + k] = o;
}

// Operands of one matrix-core launch: the table (nullptr: the exponentials
// are formed in registers from the node coefficients), the node coefficients
// of the register form, the power tables.
template <typename T>
struct SommOps {
  const typename Mfma<T>::C *E;
  const double4 *gco;
  const double2 *Vp, *Vs;
};

template <typename T, int NU, int NT, int RB>
static void agg_go(const ems_handle *h, int nrhs, int per, const SommOps<T> &o, hipStream_t st,
                   const int *cut) {
  const dim3 grid((h->q + 64 * NT - 1) / (64 * NT), h->agg_chunks, 2 * ((nrhs + RB - 1) / RB));
  const int nm = 2 * pm_bucket(h->pmax) + 1;
  if (o.E)
    hipLaunchKernelGGL((somm_aggregate_mfma_kernel<T, NU, NT, RB, false>), grid, dim3(256), 0, st,
                       h->n, h->q, nm, nrhs, reinterpret_cast<const typename Mfma<T>::C *>(h->d_xpad),
                       o.Vp, o.Vs, h->d_agg, h->agg_chunks, per,
                       o.E, cut, o.gco, h->d_xys);
  else
    hipLaunchKernelGGL((somm_aggregate_mfma_kernel<T, NU, NT, RB, true>), grid, dim3(256), 0, st,
                       h->n, h->q, nm, nrhs, reinterpret_cast<const typename Mfma<T>::C *>(h->d_xpad),
                       o.Vp, o.Vs, h->d_agg, h->agg_chunks, per,
                       o.E, cut, o.gco, h->d_xys);
}
template <typename T, int NU>
static void agg_cand(const ems_handle *h, int idx, int nrhs, int per, const SommOps<T> &o,
                     hipStream_t st, const int *cut) {
  constexpr int P = std::is_same<T, float>::value ? 1 : 0;
  switch (idx) {
    case 0: agg_go<T, NU, kCand[0][P][0][0], kCand[0][P][0][1]>(h, nrhs, per, o, st, cut); break;
    case 1: agg_go<T, NU, kCand[0][P][1][0], kCand[0][P][1][1]>(h, nrhs, per, o, st, cut); break;
    case 2: agg_go<T, NU, kCand[0][P][2][0], kCand[0][P][2][1]>(h, nrhs, per, o, st, cut); break;
    default: agg_go<T, NU, kCand[0][P][3][0], kCand[0][P][3][1]>(h, nrhs, per, o, st, cut); break;
  }
}
template <typename T, int NU, int NT, int RB>
static void dis_go(const ems_handle *h, int nrhs, int per, const SommOps<T> &o, hipStream_t st,
                   const int *cut) {
  const dim3 grid((h->n + 64 * NT - 1) / (64 * NT), h->dis_chunks, 2 * ((nrhs + RB - 1) / RB));
  const int nm = 2 * pm_bucket(h->pmax) + 1;
  if (o.E)
    hipLaunchKernelGGL((somm_disaggregate_mfma_kernel<T, NU, NT, RB, false>), grid, dim3(256), 0,
                       st, h->n, h->q, nm, nrhs, h->d_p, h->d_off,
                       reinterpret_cast<const typename Mfma<T>::C *>(h->d_bpad),
                       reinterpret_cast<typename Mfma<T>::C *>(h->d_dis), h->ncoef,
                       h->dis_chunks, per, o.E, h->d_sperm, (const int2 *)cut, o.gco, h->d_xys);
  else
    hipLaunchKernelGGL((somm_disaggregate_mfma_kernel<T, NU, NT, RB, true>), grid, dim3(256), 0,
                       st, h->n, h->q, nm, nrhs, h->d_p, h->d_off,
                       reinterpret_cast<const typename Mfma<T>::C *>(h->d_bpad),
                       reinterpret_cast<typename Mfma<T>::C *>(h->d_dis), h->ncoef,
                       h->dis_chunks, per, o.E, h->d_sperm, (const int2 *)cut, o.gco, h->d_xys);
}
template <typename T, int NU>
static void dis_cand(const ems_handle *h, int idx, int nrhs, int per, const SommOps<T> &o,
                     hipStream_t st, const int *cut) {
  constexpr int P = std::is_same<T, float>::value ? 1 : 0;
  switch (idx) {
    case 0: dis_go<T, NU, kCand[1][P][0][0], kCand[1][P][0][1]>(h, nrhs, per, o, st, cut); break;
    case 1: dis_go<T, NU, kCand[1][P][1][0], kCand[1][P][1][1]>(h, nrhs, per, o, st, cut); break;
    case 2: dis_go<T, NU, kCand[1][P][2][0], kCand[1][P][2][1]>(h, nrhs, per, o, st, cut); break;
    default: dis_go<T, NU, kCand[1][P][3][0], kCand[1][P][3][1]>(h, nrhs, per, o, st, cut); break;
  }
}

// Node coefficients of the register form: variant v (0 forward aggregate,
// 1 adjoint aggregate, 2 forward disaggregate, 3 adjoint disaggregate),
// wave type w, laid out [v][w][q].
static const double4 *gen_coef(const ems_handle *h, int v) {
  return h->d_gco ? h->d_gco + (size_t)v * 2 * h->q : nullptr;
}

// Each form reads its tables when they were built and forms the
// exponentials in registers otherwise.
bool somm_mfma_ready(const ems_handle *h, bool adjoint) {
  if (h->d_gco) return true;
  return adjoint ? (h->d_EaggA && h->d_EdisA) : (h->d_Eagg && h->d_Edis);
}

bool somm_mfma_fp32(const ems_handle *h) {
  if (h->somm_fp64) return false;
  return h->d_gco || (h->d_Eagg32 && h->d_Edis32);
}

// Matrix-core aggregate with the candidate idx (prec 0 FP64, 1 FP32; adj:
// the adjoint's conjugated factors, FP64).
hipError_t launch_somm_aggregate_mfma(const ems_handle *h, const double2 *x, int nrhs, int prec,
                                      int idx, hipStream_t st, bool adj, const int *cut) {
  if (!cut) cut = h->d_kcut;
  const int per = (h->n + h->agg_chunks - 1) / h->agg_chunks;
  const int nm = 2 * pm_bucket(h->pmax) + 1, nu = (nm + 15) / 16;
  if (adj) prec = 0;
  if (!somm_mfma_ready(h, adj) || (prec == 1 && !somm_mfma_fp32(h))) return hipErrorInvalidValue;
  const double4 *gco = gen_coef(h, adj ? 1 : 0);
  const double2 *Vp = adj ? h->d_VpA_agg : h->d_Vp, *Vs = adj ? h->d_VsA_agg : h->d_Vs;
  const SommOps<double> o64{adj ? h->d_EaggA : h->d_Eagg, gco, Vp, Vs};
  const SommOps<float> o32{h->d_Eagg32, gco, Vp, Vs};
  if (nrhs > h->ws_nrhs || !h->d_xpad) return hipErrorInvalidValue;
  {
    const int nw = 16 * nu;
    const dim3 grid((unsigned)(((int64_t)h->n * nw + 255) / 256), 2, nrhs);
    if (prec == 1)
      hipLaunchKernelGGL(somm_xpad_kernel<float2>, grid, dim3(256), 0, st, h->n,
                         pm_bucket(h->pmax), nw, h->d_p, h->d_off, x, h->ncoef, h->d_sperm,
                         reinterpret_cast<float2 *>(h->d_xpad));
    else
      hipLaunchKernelGGL(somm_xpad_kernel<double2>, grid, dim3(256), 0, st, h->n,
                         pm_bucket(h->pmax), nw, h->d_p, h->d_off, x, h->ncoef, h->d_sperm,
                         h->d_xpad);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
#define EMS_AGGM_NU(NUV)                                                                     \
  if (nu == NUV) {                                                                           \
    if (prec == 1) agg_cand<float, NUV>(h, idx, nrhs, per, o32, st, cut);                   \
    else agg_cand<double, NUV>(h, idx, nrhs, per, o64, st, cut);                            \
    return hipGetLastError();                                                                \
  }
  EMS_AGGM_NU(1)
  EMS_AGGM_NU(2)
  EMS_AGGM_NU(3)
  return hipErrorInvalidValue;
}

hipError_t launch_somm_disaggregate_mfma(const ems_handle *h, int nrhs, int prec, int idx,
                                         hipStream_t st, bool adj, const int *cut) {
  if (!cut) cut = h->d_jr;
  const int per = (h->q + h->dis_chunks - 1) / h->dis_chunks;
  const int nm = 2 * pm_bucket(h->pmax) + 1, nu = (nm + 15) / 16;
  if (adj) prec = 0;
  if (!somm_mfma_ready(h, adj) || (prec == 1 && !somm_mfma_fp32(h))) return hipErrorInvalidValue;
  const double4 *gco = gen_coef(h, adj ? 3 : 2);
  const double2 *Vp = adj ? h->d_VpA_dis : h->d_Vp, *Vs = adj ? h->d_VsA_dis : h->d_Vs;
  const SommOps<double> o64{adj ? h->d_EdisA : h->d_Edis, gco, Vp, Vs};
  const SommOps<float> o32{h->d_Edis32, gco, Vp, Vs};
  if (nrhs > h->ws_nrhs || !h->d_bpad) return hipErrorInvalidValue;
  {
    const int nw = 16 * nu;
    const dim3 grid((unsigned)(((int64_t)h->q * nw + 255) / 256), 2, nrhs);
    if (prec == 1)
      hipLaunchKernelGGL(somm_bpad_kernel<float2>, grid, dim3(256), 0, st, h->q, nm, nw,
                         h->d_refl, Vp, Vs, reinterpret_cast<float2 *>(h->d_bpad));
    else
      hipLaunchKernelGGL(somm_bpad_kernel<double2>, grid, dim3(256), 0, st, h->q, nm, nw,
                         h->d_refl, Vp, Vs, h->d_bpad);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
#define EMS_DISM_NU(NUV)                                                                     \
  if (nu == NUV) {                                                                           \
    if (prec == 1) dis_cand<float, NUV>(h, idx, nrhs, per, o32, st, cut);                   \
    else dis_cand<double, NUV>(h, idx, nrhs, per, o64, st, cut);                            \
    return hipGetLastError();                                                                \
  }
  EMS_DISM_NU(1)
  EMS_DISM_NU(2)
  EMS_DISM_NU(3)
  return hipErrorInvalidValue;
}

// The tuned (or default) candidate for a kernel, precision and batch size.
static int pick(const ems_handle *h, int kernel, int prec, int nrhs) {
  const int v = h->mfma_cfg[kernel][prec][nrhs > 1 ? 1 : 0];
  if (v >= 0) return v;
  // defaults from the tile sweep at 20000 particles, p = 15
  static constexpr int def[2][2][2] = {{{1, 2}, {1, 2}}, {{1, 2}, {1, 2}}};
  return def[kernel][prec][nrhs > 1 ? 1 : 0];
}

hipError_t launch_somm_aggregate(const ems_handle *h, const double2 *x, int nrhs, bool adjoint,
                                 bool mixed, hipStream_t st, const int *cut) {
  const int per = (h->n + h->agg_chunks - 1) / h->agg_chunks;
  const int pb = pm_bucket(h->pmax);
  const bool uni = h->p_uniform && pb == h->pmax;
  if (somm_mfma_ready(h, adjoint)) {
    const int prec = (!adjoint && mixed && somm_mfma_fp32(h)) ? 1 : 0;
    return launch_somm_aggregate_mfma(h, x, nrhs, prec, pick(h, 0, prec, nrhs), st, adjoint, cut);
  }
  dim3 grid((h->q + 255) / 256, h->agg_chunks, 2 * nrhs);
  const int mode = adjoint ? 2 : 1;
  switch (pb) {
    EMS_AGG_CASE(4)
    EMS_AGG_CASE(8)
    EMS_AGG_CASE(10)
    EMS_AGG_CASE(12)
    EMS_AGG_CASE(15)
    EMS_AGG_CASE(16)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_somm_reflect(const ems_handle *h, int nrhs, bool adjoint, hipStream_t st,
                               bool transmit) {
  dim3 grid((h->q + 255) / 256, nrhs);
  // transmit: the substrate's upgoing potentials (T in place of R)
  hipLaunchKernelGGL(somm_reflect_kernel, grid, dim3(256), 0, st, h->q, h->agg_chunks, h->d_agg,
                     h->d_w, h->d_sp, h->d_ss, transmit ? h->d_Tu : h->d_R, h->d_refl,
                     adjoint ? 1 : 0);
  return hipGetLastError();
}

#define EMS_DIS_LAUNCH(PMV, TABV)                                                          \
  hipLaunchKernelGGL((somm_disaggregate_kernel<PMV, TABV>), grid, dim3(256), 0, st, h->n, h->q, \
                     h->pmax, h->d_xy, h->d_p, h->d_off, h->d_xi, h->d_sp, h->d_ss, h->d_Vp,    \
                     h->d_Vs, h->d_refl, h->d_dis, h->ncoef, h->dis_chunks, per,               \
                     adjoint ? 1 : 0)
#define EMS_DIS_CASE(PMV)                                                                  \
  case PMV:                                                                                \
    if (mode == 1) EMS_DIS_LAUNCH(PMV, 1);                                                 \
    else EMS_DIS_LAUNCH(PMV, 2);                                                           \
    break;

// The disaggregate's split-K partial sums are complex64 exactly when the FP32
// matrix-core kernel writes them (the combine reads them by the same rule).
bool somm_dis_c64(const ems_handle *h, bool adjoint, bool mixed) {
  return somm_mfma_ready(h, adjoint) && !adjoint && mixed && somm_mfma_fp32(h);
}

hipError_t launch_somm_disaggregate(const ems_handle *h, int nrhs, bool adjoint, bool mixed,
                                    hipStream_t st, const int *cut) {
  const int per = (h->q + h->dis_chunks - 1) / h->dis_chunks;
  if (somm_mfma_ready(h, adjoint)) {
    const int prec = somm_dis_c64(h, adjoint, mixed) ? 1 : 0;
    return launch_somm_disaggregate_mfma(h, nrhs, prec, pick(h, 1, prec, nrhs), st, adjoint, cut);
  }
  dim3 grid((h->n + 255) / 256, h->dis_chunks, 2 * nrhs);
  const int mode = adjoint ? 2 : 1;
  switch (pm_bucket(h->pmax)) {
    EMS_DIS_CASE(4)
    EMS_DIS_CASE(8)
    EMS_DIS_CASE(10)
    EMS_DIS_CASE(12)
    EMS_DIS_CASE(15)
    EMS_DIS_CASE(16)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Tables of the geometry-dependent exponentials (set-up, once per geometry
// and frequency):  Eagg[w][m][j] = e^{s_w(j) y_m - i xi_j x_m},
// Edis[w][j][l] = e^{i xi_j x_l + s_w(j) y_l}, with m and l the positions of
// the particles in depth order (sperm maps them to particle indices).
__global__ void etab_agg_kernel(int n, int q, const double *__restrict__ xy,
                                const int *__restrict__ sperm, const double2 *__restrict__ xi_t,
                                const double2 *__restrict__ sp_t, const double2 *__restrict__ ss_t,
                                double2 *__restrict__ E, float2 *__restrict__ E32,
                                double2 *__restrict__ EA) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  const int w = blockIdx.z;
  if (j >= q) return;
  const double2 xi = xi_t[j];
  const double2 s = w ? ss_t[j] : sp_t[j];
  const int mo = sperm[m];
  const double xm = xy[2 * mo], ym = xy[2 * mo + 1];
  // s y - i xi x
  const double2 e = cexp(make_double2(s.x * ym + xi.y * xm, s.y * ym - xi.x * xm));
  const int64_t at = ((int64_t)w * n + m) * q + j;
  E[at] = e;
  if (E32) E32[at] = make_float2((float)e.x, (float)e.y);
  // adjoint aggregate table: conj(e^{i xi x_m + s y_m}) in this layout
  if (EA) EA[at] = cconj(cexp(make_double2(s.x * ym - xi.y * xm, s.y * ym + xi.x * xm)));
}

__global__ void etab_dis_kernel(int n, int q, const double *__restrict__ xy,
                                const int *__restrict__ sperm, const double2 *__restrict__ xi_t,
                                const double2 *__restrict__ sp_t, const double2 *__restrict__ ss_t,
                                double2 *__restrict__ E, float2 *__restrict__ E32,
                                double2 *__restrict__ EA) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int w = blockIdx.z;
  if (l >= n) return;
  const double2 xi = xi_t[j];
  const double2 s = w ? ss_t[j] : sp_t[j];
  const int lo = sperm[l];
  const double xl = xy[2 * lo], yl = xy[2 * lo + 1];
  // i xi x + s y
  const double2 e = cexp(make_double2(s.x * yl - xi.y * xl, s.y * yl + xi.x * xl));
  const int64_t at = ((int64_t)w * q + j) * n + l;
  E[at] = e;
  if (E32) E32[at] = make_float2((float)e.x, (float)e.y);
  // adjoint disaggregate table: conj(e^{s y_l - i xi x_l}) in this layout
  if (EA) EA[at] = cconj(cexp(make_double2(s.x * yl + xi.y * xl, s.y * yl - xi.x * xl)));
}

// Node coefficients g of E = exp((g.x y + g.y x) + i (g.z y + g.w x)) for
// the register form, [variant][wave][q] (variants as in gen_coef), and the
// particle positions in depth order.  With s = s_w(j), xi = xi_j:
//   forward aggregate    s y - i xi x                 g = ( s_r,  xi_i,  s_i, -xi_r)
//   adjoint aggregate    conj(i xi x + s y)           g = ( s_r, -xi_i, -s_i, -xi_r)
//   forward disaggregate i xi x + s y                 g = ( s_r, -xi_i,  s_i,  xi_r)
//   adjoint disaggregate conj(s y - i xi x)           g = ( s_r,  xi_i, -s_i,  xi_r)
// (the same four factors as the tables etab_agg_kernel / etab_dis_kernel).
__global__ void gen_coef_kernel(int n, int q, const double *__restrict__ xy,
                                const int *__restrict__ sperm, const double2 *__restrict__ xi_t,
                                const double2 *__restrict__ sp_t, const double2 *__restrict__ ss_t,
                                double4 *__restrict__ gco, double2 *__restrict__ xys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int o = sperm[i];
    xys[i] = make_double2(xy[2 * o], xy[2 * o + 1]);
  }
  if (i >= 2 * q) return;
  const int w = i / q, j = i - w * q;
  const double2 xi = xi_t[j];
  const double2 s = w ? ss_t[j] : sp_t[j];
  const size_t V = (size_t)2 * q;
  gco[i] = make_double4(s.x, xi.y, s.y, -xi.x);
  gco[V + i] = make_double4(s.x, -xi.y, -s.y, -xi.x);
  gco[2 * V + i] = make_double4(s.x, -xi.y, s.y, xi.x);
  gco[3 * V + i] = make_double4(s.x, xi.y, -s.y, xi.x);
}

hipError_t launch_gen_coef(ems_handle *h, hipStream_t st) {
  const int m = std::max(h->n, 2 * h->q);
  hipLaunchKernelGGL(gen_coef_kernel, dim3((m + 255) / 256), dim3(256), 0, st, h->n, h->q, h->d_xy,
                     h->d_sperm, h->d_xi, h->d_sp, h->d_ss, h->d_gco, h->d_xys);
  return hipGetLastError();
}

hipError_t launch_etables(ems_handle *h, hipStream_t st) {
  hipLaunchKernelGGL(etab_agg_kernel, dim3((h->q + 255) / 256, h->n, 2), dim3(256), 0, st, h->n,
                     h->q, h->d_xy, h->d_sperm, h->d_xi, h->d_sp, h->d_ss, h->d_Eagg,
                     h->d_Eagg32, h->d_EaggA);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(etab_dis_kernel, dim3((h->n + 255) / 256, h->q, 2), dim3(256), 0, st, h->n,
                     h->q, h->d_xy, h->d_sperm, h->d_xi, h->d_sp, h->d_ss, h->d_Edis,
                     h->d_Edis32, h->d_EdisA);
  return hipGetLastError();
}

}  // namespace ems
