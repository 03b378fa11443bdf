// Dense block operations of the block Krylov solver on the matrix cores
// (FP64 16x16x4 MFMA, complex products as four real ones):
//
//   bdot:   H[i][c] = sum_r conj(V_i[r]) W_c[r]        (k x s, i < k, c < s <= 64)
//   baxpy:  out_c[r] = beta out_c[r] + alpha sum_i V_i[r] H[i][c]
//
// V holds k vectors and W (or out) s vectors of length n, each contiguous
// (vector i at V + i n).  bdot splits the long index r into chunks whose
// partial products are summed in a fixed order by bdot_reduce_kernel, so
// results are reproducible run to run.  A wavefront owns 16 rows (i, or r)
// by all 64 columns c (four 16-column tiles); the four wavefronts of a
// workgroup share the column operand through the L1 cache.
#include <algorithm>

#include "dev.h"
#include "ems_internal.h"

namespace ems {

typedef double blk_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ blk_d4 blk_mf(double a, double b, blk_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kBlkCols = 64;  // largest block size s

// part[chunk][i][c] over r in the chunk; lane (i16, kq): A entry (row i16 =
// basis vector, K index kq = r), B entry (K index kq = r, column i16 + 16 t).
__global__ __launch_bounds__(256) void bdot_kernel(const double2 *__restrict__ V, int k,
                                                   const double2 *__restrict__ W, int s,
                                                   int64_t n, int64_t per_chunk,
                                                   double2 *__restrict__ part) {
  const int lane = threadIdx.x & 63, kq = lane >> 4, i16 = lane & 15;
  const int i0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (i0 >= k) return;  // whole wavefront; no barrier in the kernel
  const int chunk = blockIdx.y;
  const int64_t r0 = (int64_t)chunk * per_chunk, r1 = min(n, r0 + per_chunk);
  const int iv = min(i0 + i16, k - 1);
  const double2 *Vi = V + (int64_t)iv * n;
  const double2 *Wc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) Wc[t] = W + (int64_t)min(16 * t + i16, s - 1) * n;
  blk_d4 ar[4], ai[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) ar[t] = ai[t] = blk_d4{0, 0, 0, 0};
  double2 a = make_double2(0.0, 0.0), b[4];
  auto fetch = [&](int64_t r) {
    const bool ok = r + kq < r1;
    const int64_t rr = ok ? r + kq : r0;
    a = ok ? Vi[rr] : make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < 4; ++t) b[t] = ok ? Wc[t][rr] : make_double2(0.0, 0.0);
  };
  if (r0 < r1) fetch(r0);
  for (int64_t r = r0; r < r1; r += 4) {
    const double vr = a.x, vi = a.y;
    double br[4], bi[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      br[t] = b[t].x;
      bi[t] = b[t].y;
    }
    fetch(r + 4);
    // conj(v) w = (vr wr + vi wi) + i (vr wi - vi wr)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ar[t] = blk_mf(vr, br[t], ar[t]);
      ai[t] = blk_mf(vr, bi[t], ai[t]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ar[t] = blk_mf(vi, bi[t], ar[t]);
      ai[t] = blk_mf(-vi, br[t], ai[t]);
    }
  }
  // accumulator element v: row i0 + kq + 4 v, column 16 t + i16
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = 16 * t + i16;
    if (c >= s) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + kq + 4 * v;
      if (i < k) part[((int64_t)chunk * k + i) * s + c] = make_double2(ar[t][v], ai[t][v]);
    }
  }
}

__global__ void bdot_reduce_kernel(const double2 *__restrict__ part, int chunks, int64_t ks,
                                   double2 *__restrict__ H) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ks) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int c = 0; c < chunks; ++c) acc = cadd(acc, part[(int64_t)c * ks + e]);
  H[e] = acc;
}

// out_c[r] = beta out_c[r] + alpha sum_i V_i[r] H[i][c]; lane (i16, kq): A
// entry (row i16 = r, K index kq = i), B entry (K index kq = i, column i16 + 16 t).
__global__ __launch_bounds__(256) void baxpy_kernel(const double2 *__restrict__ V, int k,
                                                    const double2 *__restrict__ H, int s,
                                                    int64_t n, double2 *__restrict__ out,
                                                    double alpha, double beta) {
  const int lane = threadIdx.x & 63, kq = lane >> 4, i16 = lane & 15;
  const int64_t rb = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (rb >= n) return;
  const int64_t rr = min(rb + i16, n - 1);
  blk_d4 ar[4], ai[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) ar[t] = ai[t] = blk_d4{0, 0, 0, 0};
  double2 a = make_double2(0.0, 0.0), b[4];
  auto fetch = [&](int i) {
    const bool ok = i + kq < k;
    const int ii = ok ? i + kq : 0;
    a = ok ? V[(int64_t)ii * n + rr] : make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = 16 * t + i16;
      b[t] = (ok && c < s) ? H[(int64_t)ii * s + c] : make_double2(0.0, 0.0);
    }
  };
  fetch(0);
  for (int i = 0; i < k; i += 4) {
    const double vr = a.x, vi = a.y;
    double br[4], bi[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      br[t] = b[t].x;
      bi[t] = b[t].y;
    }
    fetch(i + 4);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ar[t] = blk_mf(vr, br[t], ar[t]);
      ai[t] = blk_mf(vr, bi[t], ai[t]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ar[t] = blk_mf(-vi, bi[t], ar[t]);
      ai[t] = blk_mf(vi, br[t], ai[t]);
    }
  }
  // accumulator element v: row r = rb + kq + 4 v, column 16 t + i16
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = 16 * t + i16;
    if (c >= s) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t r = rb + kq + 4 * v;
      if (r >= n) continue;
      double2 *o = out + (int64_t)c * n + r;
      const double2 prev = beta != 0.0 ? *o : make_double2(0.0, 0.0);
      *o = make_double2(beta * prev.x + alpha * ar[t][v], beta * prev.y + alpha * ai[t][v]);
    }
  }
}

int bdot_chunks(int k, int64_t n) {
  const int waves = (k + 15) / 16;
  int c = std::max(1, std::min(512, (2048 + waves - 1) / waves));
  return (int)std::min<int64_t>(c, std::max<int64_t>(1, n / 64));
}

hipError_t launch_bdot(const double2 *V, int k, const double2 *W, int s, int64_t n, double2 *H,
                       double2 *part, hipStream_t st) {
  if (k <= 0 || s <= 0 || s > kBlkCols || n <= 0) return hipErrorInvalidValue;
  const int chunks = bdot_chunks(k, n);
  const int64_t per = (n + chunks - 1) / chunks;
  hipLaunchKernelGGL(bdot_kernel, dim3((k + 63) / 64, chunks), dim3(256), 0, st, V, k, W, s, n,
                     per, part);
  const int64_t ks = (int64_t)k * s;
  hipLaunchKernelGGL(bdot_reduce_kernel, dim3((unsigned)((ks + 255) / 256)), dim3(256), 0, st, part,
                     chunks, ks, H);
  return hipGetLastError();
}

hipError_t launch_baxpy(const double2 *V, int k, const double2 *H, int s, int64_t n,
                        double2 *out, double alpha, double beta, hipStream_t st) {
  if (k <= 0 || s <= 0 || s > kBlkCols || n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(baxpy_kernel, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, st, V, k, H, s,
                     n, out, alpha, beta);
  return hipGetLastError();
}

}  // namespace ems
