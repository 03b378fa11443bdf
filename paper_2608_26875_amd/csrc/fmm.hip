// Batched Toeplitz products for the free-space FMM: P2M, M2M, M2L (+L2L)
// and L2P are all out_k = sum_j s_{j-k} in_j with a tabulated symbol s (see
// fmm.cpp).  One workgroup owns one output expansion (or a 192-row chunk of
// it) and sweeps the tasks that feed it, so every output is written by exactly
// one workgroup (no atomics, fixed summation order).  The symbol window the
// chunk needs is staged in LDS; each lane forms R output coefficients from it
// and from the input vector read with scalar loads (see below).  Right-hand
// sides are taken 8 at a time, the symbol window of a task staged once for
// all of them.
#include <algorithm>

#include "dev.h"
#include "ems_internal.h"

namespace ems {

// One wavefront per item; lane t owns the R consecutive output rows
// k_lo + R t + r.  For a fixed column j the symbols of those rows are
// s_{j-k}, consecutive entries of the staged window, so a lane keeps a ring
// of R of them and reads one new entry per column: one LDS read (stride R
// entries across lanes, conflict-free for odd R) per R complex multiply-adds.
// The input coefficient of column j is the same for every lane and is read
// with scalar loads straight from the expansion array.
// Launches whose outputs all have at most 64 rows (the particle-side L2P of
// orders up to 31) take R = 1, one row per lane: with R = 3 only a third of
// the lanes would hold rows.
constexpr int kToepR = 3;
constexpr int kToepRows = 64 * kToepR;
static_assert(kToepRows == kFmmRows, "item chunk of the plan");

template <int RB, int R>
__global__ __launch_bounds__(64) void toep_task_kernel(
    const int *__restrict__ ptr, const int64_t *__restrict__ in_base,
    const int *__restrict__ in_P, const int64_t *__restrict__ sym_base,
    const int *__restrict__ sym_L, const int *__restrict__ sgn,
    const int64_t *__restrict__ out_base, const int *__restrict__ out_P,
    const int *__restrict__ item_out, const int *__restrict__ item_row0,
    const int *__restrict__ item_t0, const int *__restrict__ item_t1,
    const int *__restrict__ item_slot, const double2 *__restrict__ in_main, int64_t in_stride,
    const double2 *__restrict__ in_alt, int64_t alt_stride, const double2 *__restrict__ pool,
    double2 *__restrict__ out, int64_t out_stride, double2 *__restrict__ part,
    int64_t part_stride, int accumulate, int max_in, int nrhs) {
  constexpr int ROWSR = 64 * R;            // rows of one item
  extern __shared__ double2 vs[];           // [2 max_in + kToepRows]
  const int item = blockIdx.x, r0 = blockIdx.y * RB, tid = threadIdx.x;
  const int o = item_out[item], row0 = item_row0[item];
  const int Po = out_P[o];
  const int rows = min(ROWSR, 2 * Po + 1 - row0);
  const int k_lo = -Po + row0, k_hi = k_lo + rows - 1;
  const int kb = k_lo + tid * R;            // first row of this lane
  const int b0 = k_hi - kb;                 // rows r <= b0 are inside the item
  double2 acc[RB][R];
#pragma unroll
  for (int rr = 0; rr < RB; ++rr)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[rr][r] = make_double2(0.0, 0.0);
  const int slot = item_slot[item];
  for (int t = item_t0[item]; t < item_t1[item]; ++t) {
    const int Pi = in_P[t], L = sym_L[t], sg = sgn[t];
    const int nin = 2 * Pi + 1;
    // window vs[e] = s_{nlo + e}, nlo = -Pi - k_hi (entry of column j, row k: j + Pi + k_hi - k)
    const int nlo = -Pi - k_hi;
    const int cnt = 2 * Pi + rows;
    const double2 *sym = pool + sym_base[t] + L;
    __syncthreads();
    for (int e = tid; e < cnt; e += 64) {
      const int nu = nlo + e;
      double2 v = sym[nu];
      if (sg == -1 && (nu & 1)) v = make_double2(-v.x, -v.y);
      vs[e] = v;
    }
    __syncthreads();
    if (b0 < 0) continue;                   // lane beyond the item's rows
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      if (r0 + rr >= nrhs) break;           // uniform over the wavefront
      const double2 *src =
          (sg == 2 ? in_alt + (int64_t)(r0 + rr) * alt_stride
                   : in_main + (int64_t)(r0 + rr) * in_stride) + in_base[t];
      // ring[m mod R] = window entry of (column m, row kb): vs[m + b0]
      double2 ring[R];
#pragma unroll
      for (int d = 1; d < R; ++d) ring[(R - d) % R] = vs[max(b0 - d, 0)];
      // two ring cycles per iteration (column index mod R stays compile-time)
      constexpr int U = 2 * R;
      int jj0 = 0;
      for (; jj0 + U <= nin; jj0 += U) {
#pragma unroll
        for (int d = 0; d < U; ++d) {
          ring[d % R] = vs[jj0 + d + b0];
          const double2 v = src[jj0 + d];
#pragma unroll
          for (int r = 0; r < R; ++r) cfma(acc[rr][r], ring[(d - r + U) % R], v);
        }
      }
#pragma unroll
      for (int d = 0; d < U; ++d) {
        if (jj0 + d < nin) {
          ring[d % R] = vs[jj0 + d + b0];
          const double2 v = src[jj0 + d];
#pragma unroll
          for (int r = 0; r < R; ++r) cfma(acc[rr][r], ring[(d - r + U) % R], v);
        }
      }
    }
  }
  if (b0 < 0) return;
#pragma unroll
  for (int rr = 0; rr < RB; ++rr) {
    if (r0 + rr >= nrhs) break;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r > b0) break;                    // row beyond the item
      if (slot >= 0) {                      // partial over a group of the tasks
        part[(int64_t)(r0 + rr) * part_stride + (int64_t)slot * kFmmRows + (kb + r - k_lo)] =
            acc[rr][r];
        continue;
      }
      double2 *d = out + (int64_t)(r0 + rr) * out_stride + out_base[o] + (kb + r + Po);
      if (accumulate) *d = cadd(*d, acc[rr][r]);
      else *d = acc[rr][r];
    }
  }
}

// ---------------------------------------------------------------------------
// M2L on the matrix cores (plan: M2lPlan in fmm.cpp).  One wavefront per work
// item: rows 16 rt .. 16 (rt + kM2lRowTiles) - 1 of product g (kM2lRowTiles
// row tiles of 16), the kM2lCols = 16 target boxes of one tile, over a group
// of the tile's offsets:
//   acc[k][b] += sum_j s^o_{j-k} M_{src(b,o)}[j]
// as 16x16x4 MFMAs (A = the Toeplitz symbol, B = the gathered source
// multipoles, a complex product three real MFMAs).  Lane (i16, kq) supplies A
// entry (row i16, K index kq) of each row tile and B entry (K index kq, box
// i16), which all row tiles of the item share; both are read straight from
// the symbol pool and the multipole array (L1/L2 resident), kM2lKB K steps at
// a time, the next ones loaded before the current ones are multiplied.  No LDS and no barriers: waves run independently and
// the hardware overlaps their loads.  T = double (FP64 MFMA) or float (FP32
// MFMA on rounded operands, FP32 accumulation) for the mixed form.
typedef double m2l_d4 __attribute__((ext_vector_type(4)));
typedef float m2l_f4 __attribute__((ext_vector_type(4)));
template <typename T> struct M2lM;
template <> struct M2lM<double> {
  using Acc = m2l_d4;
  __device__ static Acc mf(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int kq, int v) { return kq + 4 * v; }
};
template <> struct M2lM<float> {
  using Acc = m2l_f4;
  __device__ static Acc mf(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int kq, int v) { return 4 * kq + v; }
};

constexpr int kM2lKB = kM2lRowTiles > 1 ? 2 : 4;  // K steps of 4 loaded together

template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void m2l_mfma_kernel(
    int i0, int i1, const int *__restrict__ it_g, const int *__restrict__ it_rt,
    const int *__restrict__ it_tile, const int *__restrict__ it_e0,
    const int *__restrict__ it_e1, const int *__restrict__ it_slot,
    const int *__restrict__ g_P, const int *__restrict__ g_nb, const int64_t *__restrict__ g_off,
    const int64_t *__restrict__ g_poff, const int *__restrict__ tile_box,
    const int64_t *__restrict__ ent_sym, const int *__restrict__ ent_src,
    const double2 *__restrict__ pool, const double2 *__restrict__ mult, double2 *__restrict__ loc,
    int64_t stride, double2 *__restrict__ part, int64_t pstride) {
  using Acc = typename M2lM<T>::Acc;
  const int it = i0 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (it >= i1) return;  // whole wavefront; the kernel has no barrier
  const int lane = threadIdx.x & 63, kq = lane >> 4, i16 = lane & 15;
  const int g = it_g[it], P = g_P[g], N = 2 * P + 1;
  const int row0 = 16 * it_rt[it], tile = it_tile[it];
  const int r = blockIdx.y;
  const double2 *M = mult + (int64_t)r * stride + g_off[g];
  constexpr int RT = kM2lRowTiles;
  // row tiles of the item inside the product (uniform over the wave)
  const int nrt = min(RT, (N - row0 + 15) / 16);
  // 3M complex products: K1 += (Ar + Ai) Br, K2 += Ar (Bi - Br),
  // K3 += Ai (Br + Bi); Re = K1 - K3, Im = K1 + K2 after the loop.
  Acc k1[RT], k2[RT], k3[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) k1[t] = k2[t] = k3[t] = Acc{0, 0, 0, 0};
  const int krow = row0 + i16;  // A row of this lane in the first row tile
  const int e0 = it_e0[it], e1 = it_e1[it];
  // The operand stream runs over (entry, chunk of kM2lKB K steps) without a
  // break between entries: the last chunk of an entry loads the first chunk
  // of the next one, whose symbol offset and source box are loaded one
  // entry ahead.
  auto entry = [&](int e, const double2 *&sym, const double2 *&Mb, bool &live) {
    const int ee = min(e, e1 - 1);
    sym = pool + ent_sym[ee];
    const int sb = ent_src[(int64_t)ee * kM2lCols + i16];
    live = sb >= 0;
    Mb = M + (int64_t)(sb < 0 ? 0 : sb) * N;
  };
  auto load = [&](const double2 *sym, const double2 *Mb, bool live, int j0,
                  double2 (&a)[RT][kM2lKB], double2 (&b)[kM2lKB]) {
#pragma unroll
    for (int u = 0; u < kM2lKB; ++u) {
      const int jj = j0 + 4 * u + kq;
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        // rows past the product are never stored; the clamp keeps their
        // reads inside the symbol
        const int nu = min(max(jj - krow - 16 * t, -2 * P), 2 * P);
        a[t][u] = t < nrt ? sym[nu] : make_double2(0.0, 0.0);
      }
      b[u] = (live && jj < N) ? Mb[jj] : make_double2(0.0, 0.0);
    }
  };
  if (e0 < e1) {
    const double2 *symc, *Mbc, *symn, *Mbn;
    bool livec, liven;
    entry(e0, symc, Mbc, livec);
    entry(e0 + 1, symn, Mbn, liven);
    double2 ca[RT][kM2lKB], cb[kM2lKB], na[RT][kM2lKB], nb[kM2lKB];
    load(symc, Mbc, livec, 0, ca, cb);
    for (int e = e0; e < e1; ++e) {
      for (int j0 = 0; j0 < N; j0 += 4 * kM2lKB) {
        if (j0 + 4 * kM2lKB < N) load(symc, Mbc, livec, j0 + 4 * kM2lKB, na, nb);
        else if (e + 1 < e1) load(symn, Mbn, liven, 0, na, nb);
#pragma unroll
        for (int u = 0; u < kM2lKB; ++u) {
          if (j0 + 4 * u >= N) break;  // K steps past 2P+1 (uniform over the wave)
          const T bre = (T)cb[u].x, bim = (T)cb[u].y, bd = bim - bre, bs = bre + bim;
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            if (t >= nrt) break;  // uniform over the wave
            const T are = (T)ca[t][u].x, aim = (T)ca[t][u].y;
            k1[t] = M2lM<T>::mf(are + aim, bre, k1[t]);
            k2[t] = M2lM<T>::mf(are, bd, k2[t]);
            k3[t] = M2lM<T>::mf(aim, bs, k3[t]);
          }
        }
#pragma unroll
        for (int u = 0; u < kM2lKB; ++u) {
#pragma unroll
          for (int t = 0; t < RT; ++t) ca[t][u] = na[t][u];
          cb[u] = nb[u];
        }
      }
      symc = symn;
      Mbc = Mbn;
      livec = liven;
      entry(e + 2, symn, Mbn, liven);
    }
  }
  // accumulator element v of row tile t: row 16 t + M2lM::row(kq, v), box column i16
  const int b = tile_box[(int64_t)tile * kM2lCols + i16];
  if (b < 0) return;
  const int slot = it_slot[it];
  double2 *dst = slot < 0 ? loc + (int64_t)r * stride + g_off[g] + (int64_t)b * N
                          : part + (int64_t)r * pstride + g_poff[g] +
                                ((int64_t)slot * g_nb[g] + b) * N;
#pragma unroll
  for (int t = 0; t < RT; ++t) {
    const Acc ar = k1[t] - k3[t], ai = k1[t] + k2[t];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = row0 + 16 * t + M2lM<T>::row(kq, v);
      if (k < N) dst[k] = make_double2((double)ar[v], (double)ai[v]);
    }
  }
}

// L_b = sum of the G partial slots of product g, in slot order.
__global__ __launch_bounds__(256) void m2l_reduce_kernel(int G, int nb, int N, int64_t off,
                                                         int64_t poff, const double2 *__restrict__ part,
                                                         int64_t pstride, double2 *__restrict__ loc,
                                                         int64_t stride) {
  const int64_t tot = (int64_t)nb * N;
  const int r = blockIdx.y;
  const double2 *pp = part + (int64_t)r * pstride + poff;
  double2 *L = loc + (int64_t)r * stride + off;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (int64_t)gridDim.x * 256) {
    double2 s = make_double2(0.0, 0.0);
    for (int g = 0; g < G; ++g) s = cadd(s, pp[(int64_t)g * tot + i]);
    L[i] = s;
  }
}

// M2L of tree level li for both waves; mixed: FP32 matrix cores for the
// products whose symbols stay inside FP32's range (largest |s| below 1e30).
hipError_t launch_m2l_mfma(const ems_handle *h, int li, int nrhs, bool mixed, hipStream_t st) {
  const FmmPlan &F = h->fmm;
  const M2lPlan &Q = F.m2l;
  const M2lDev &D = h->m2l_dev;
  for (size_t g = 0; g < Q.g_P.size(); ++g) {
    if (Q.g_li[g] != li) continue;
    const int i0 = Q.g_item0[g], i1 = Q.g_item0[g + 1];
    if (i1 <= i0) continue;
    const dim3 grid((unsigned)((i1 - i0 + 3) / 4), nrhs);
    const bool f32 = mixed && Q.g_symmax[g] < 1e30;
#define EMS_M2L_LAUNCH(T)                                                                      \
  hipLaunchKernelGGL((m2l_mfma_kernel<T>), grid, dim3(256), 0, st, i0, i1, D.it_g, D.it_rt,    \
                     D.it_tile, D.it_e0, D.it_e1, D.it_slot, D.g_P, D.g_nb, D.g_off, D.g_poff, \
                     D.tile_box, D.ent_sym, D.ent_src, h->d_pool, h->d_mult, h->d_loc,        \
                     F.exp_len, h->d_m2l_part, Q.part_len)
    if (f32) EMS_M2L_LAUNCH(float);
    else EMS_M2L_LAUNCH(double);
#undef EMS_M2L_LAUNCH
    if (Q.g_G[g] > 1) {
      const int N = 2 * Q.g_P[g] + 1;
      const int64_t tot = (int64_t)Q.g_nb[g] * N;
      hipLaunchKernelGGL(m2l_reduce_kernel, dim3((unsigned)std::min<int64_t>(2048, (tot + 255) / 256), nrhs),
                         dim3(256), 0, st, Q.g_G[g], Q.g_nb[g], N, Q.g_off[g], Q.g_poff[g],
                         h->d_m2l_part, Q.part_len, h->d_loc, F.exp_len);
    }
  }
  return hipGetLastError();
}

// Sum of the task-group partials of one (output, chunk), in group order.
__global__ __launch_bounds__(kFmmRows) void fmm_reduce_kernel(
    const int *__restrict__ red_out, const int *__restrict__ red_row0,
    const int *__restrict__ red_slot0, const int *__restrict__ red_g,
    const int *__restrict__ out_P, const int64_t *__restrict__ out_base,
    const double2 *__restrict__ part, int64_t part_stride, double2 *__restrict__ out,
    int64_t out_stride, int accumulate) {
  const int k = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const int o = red_out[k], Po = out_P[o], row0 = red_row0[k];
  const int rows = min(kFmmRows, 2 * Po + 1 - row0);
  if (tid >= rows) return;
  const double2 *pp = part + (int64_t)r * part_stride + (int64_t)red_slot0[k] * kFmmRows + tid;
  double2 s = make_double2(0.0, 0.0);
  for (int g = 0; g < red_g[k]; ++g) s = cadd(s, pp[(int64_t)g * kFmmRows]);
  double2 *d = out + (int64_t)r * out_stride + out_base[o] + row0 + tid;
  if (accumulate) *d = cadd(*d, s);
  else *d = s;
}

hipError_t launch_fmm(const ems_handle *h, const double2 *x, double2 *fre, int nrhs, bool mixed,
                      hipStream_t st) {
  const FmmPlan &F = h->fmm;
  for (size_t li = 0; li < F.launches.size(); ++li) {
    const FmmLaunch &L = F.launches[li];
    const FmmDev &D = h->fmm_dev[li];
    if (L.gemm_level >= 0) {
      ProfScope ps(const_cast<ems_handle *>(h), L.name, st, L.flops * nrhs);
      const hipError_t e = launch_m2l_mfma(h, L.gemm_level, nrhs, mixed, st);
      if (e != hipSuccess) return e;
      continue;
    }
    const double2 *in = L.in_kind == 0 ? x : (L.in_kind == 1 ? h->d_mult : h->d_loc);
    const int64_t in_stride = L.in_kind == 0 ? h->ncoef : F.exp_len;
    double2 *out = L.out_kind == 1 ? h->d_mult : (L.out_kind == 2 ? h->d_loc : fre);
    const int64_t out_stride = L.out_kind == 3 ? h->ncoef : F.exp_len;
    const size_t lds = sizeof(double2) * (size_t)(2 * L.max_in_P + kToepRows);
    ProfScope ps(const_cast<ems_handle *>(h), L.name, st, L.flops * nrhs);
    const int64_t pst = (int64_t)F.max_slots * kFmmRows;
    const bool narrow = 2 * L.max_out_P + 1 <= 64;
#define EMS_TOEP_LAUNCH(RBV, RV)                                                               \
  hipLaunchKernelGGL((toep_task_kernel<RBV, RV>),                                              \
                     dim3((unsigned)L.item_out.size(), (nrhs + RBV - 1) / RBV), dim3(64), lds, st, \
                     D.ptr, D.in_base, D.in_P, D.sym_base, D.sym_L, D.sgn, D.out_base, D.out_P,   \
                     D.item_out, D.item_row0, D.item_t0, D.item_t1, D.item_slot, in, in_stride,   \
                     h->d_loc, F.exp_len, h->d_pool, out, out_stride, h->d_fmm_part, pst,        \
                     L.accumulate, L.max_in_P, nrhs)
    if (nrhs > 1) {
      if (narrow) EMS_TOEP_LAUNCH(8, 1);
      else EMS_TOEP_LAUNCH(8, kToepR);
    } else {
      if (narrow) EMS_TOEP_LAUNCH(1, 1);
      else EMS_TOEP_LAUNCH(1, kToepR);
    }
#undef EMS_TOEP_LAUNCH
    if (!L.red_out.empty())
      hipLaunchKernelGGL(fmm_reduce_kernel, dim3((unsigned)L.red_out.size(), nrhs), dim3(kFmmRows),
                         0, st, D.red_out, D.red_row0, D.red_slot0, D.red_g, D.out_P, D.out_base,
                         h->d_fmm_part, pst, out, out_stride, L.accumulate);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// v_m -> conj(P v_m) per particle block and wave, with (P v)_n = (-1)^n v_{-n}.
// The free-space operator is reciprocal, (T^{lm})^T = P T^{ml} P, so
// T^H v = P conj(T conj(P v)).
__global__ void conj_flip_kernel(const int *__restrict__ p, const int64_t *__restrict__ off,
                                 const double2 *__restrict__ in, double2 *__restrict__ out,
                                 int64_t ncoef) {
  const int m = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
  const int pm = p[m], N = 2 * pm + 1;
  if (lane >= 2 * N) return;
  const int w = lane < N ? 0 : 1;
  const int n = (w ? lane - N : lane) - pm;
  const int64_t b = (int64_t)r * ncoef + off[m] + w * N;
  double2 v = in[b + (-n) + pm];
  if (n & 1) v = make_double2(-v.x, -v.y);
  out[b + n + pm] = make_double2(v.x, -v.y);
}

hipError_t launch_conj_flip(const ems_handle *h, const double2 *in, double2 *out, int nrhs,
                            hipStream_t st) {
  hipLaunchKernelGGL(conj_flip_kernel, dim3(h->n, nrhs), dim3(part_threads(h)), 0, st, h->d_p, h->d_off, in, out,
                     h->ncoef);
  return hipGetLastError();
}

}  // namespace ems
