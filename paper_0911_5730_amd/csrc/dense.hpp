// Workgroup-cooperative dense FP64 routines used inside the batched kernels.
// One workgroup (kNT threads = 4 wave64) owns one small dense problem; matrices
// are column-major with an explicit leading dimension and may live in LDS or
// in global memory.  Every routine ends with a barrier so that its results are
// visible to the whole workgroup.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace bddc {

// Walks the flat indices start, start + step, ... of a column-major space with
// m rows as (row i, column j) without a division per step (integer division by
// a run-time value costs tens of instructions on the vector unit).
// With no rows the walk is empty: j starts past any column count.
struct ColWalk {
  int i, j, di, dj, m;
  __device__ ColWalk(int start, int step, int rows) : m(rows > 0 ? rows : 1) {
    i = start % m;
    j = rows > 0 ? start / m : 0x7fffffff;
    di = step % m;
    dj = rows > 0 ? step / m : 0;
  }
  __device__ void next() {
    i += di;
    j += dj;
    if (i >= m) {
      i -= m;
      ++j;
    }
  }
};


__device__ inline void flag_bad(int* status) {
  if (status) atomicOr(status, 1);
}

// Eliminate the first m columns of the symmetric n x n matrix A (lower triangle
// referenced): on exit the leading m columns hold the Cholesky factor L of the
// leading block and the rows below it (L21 = A21 L11^{-T}); the trailing
// (n-m) x (n-m) lower triangle holds the Schur complement A22 - L21 L21^T.
__device__ inline void wg_partial_potrf(double* A, int lda, int n, int m, int* status) {
  const int tid = threadIdx.x;
  for (int j = 0; j < m; ++j) {
    __syncthreads();
    double d = A[j + (size_t)j * lda];
    const bool ok = d > 0.0 && d < 1e308;
    if (!ok && tid == 0) flag_bad(status);
    const double s = ok ? sqrt(d) : 1.0;
    const double inv = 1.0 / s;
    for (int i = j + 1 + tid; i < n; i += kNT) A[i + (size_t)j * lda] *= inv;
    __syncthreads();
    if (tid == 0) A[j + (size_t)j * lda] = s;
    const int w = n - j - 1;
    for (ColWalk w_(tid, kNT, w); w_.j < w; w_.next()) {
      const int ii = w_.i, cc = w_.j;
      [[maybe_unused]] const int idx = ii + cc * w;
      if (ii >= cc) {
        const int i = j + 1 + ii, c = j + 1 + cc;
        A[i + (size_t)c * lda] -= A[i + (size_t)j * lda] * A[c + (size_t)j * lda];
      }
    }
  }
  __syncthreads();
}

__device__ inline void wg_potrf(double* A, int lda, int n, int* status) {
  wg_partial_potrf(A, lda, n, n, status);
}

// Copy the lower triangle of the n x n matrix A into its upper triangle.
__device__ inline void wg_mirror_lower(double* A, int lda, int n) {
  for (ColWalk w_(threadIdx.x, kNT, n); w_.j < n; w_.next()) {
    const int i = w_.i, c = w_.j;
    [[maybe_unused]] const int idx = i + c * n;
    if (i < c) A[i + (size_t)c * lda] = A[c + (size_t)i * lda];
  }
  __syncthreads();
}

// Solve L X = B in place (L lower n x n, B n x m), one thread per column.
__device__ inline void wg_trsm_lower(const double* L, int ldl, int n, double* B, int ldb, int m) {
  for (int c = threadIdx.x; c < m; c += kNT) {
    double* b = B + (size_t)c * ldb;
    for (int i = 0; i < n; ++i) {
      double v = b[i];
      for (int k = 0; k < i; ++k) v -= L[i + (size_t)k * ldl] * b[k];
      b[i] = v / L[i + (size_t)i * ldl];
    }
  }
  __syncthreads();
}

// Solve L^T X = B in place (L lower n x n, B n x m), one thread per column.
__device__ inline void wg_trsm_lower_trans(const double* L, int ldl, int n, double* B, int ldb, int m) {
  for (int c = threadIdx.x; c < m; c += kNT) {
    double* b = B + (size_t)c * ldb;
    for (int i = n - 1; i >= 0; --i) {
      double v = b[i];
      for (int k = i + 1; k < n; ++k) v -= L[k + (size_t)i * ldl] * b[k];
      b[i] = v / L[i + (size_t)i * ldl];
    }
  }
  __syncthreads();
}

// C = alpha * op(A) op(B) + beta * C for small matrices, one thread per entry of C.
__device__ inline void wg_gemm(bool ta, bool tb, int m, int n, int k, double alpha, const double* A,
                               int lda, const double* B, int ldb, double beta, double* C, int ldc) {
  for (ColWalk w_(threadIdx.x, kNT, m); w_.j < n; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * m;
    double acc = 0.0;
    for (int p = 0; p < k; ++p) {
      const double a = ta ? A[p + (size_t)i * lda] : A[i + (size_t)p * lda];
      const double b = tb ? B[j + (size_t)p * ldb] : B[p + (size_t)j * ldb];
      acc += a * b;
    }
    C[i + (size_t)j * ldc] = (beta == 0.0 ? 0.0 : beta * C[i + (size_t)j * ldc]) + alpha * acc;
  }
  __syncthreads();
}

// sum over j = j0, j0+step, ... < n of A[j*lda] * x[j], with eight independent
// partial sums so that eight loads of A are in flight per thread (the small
// kernels here are bound by memory latency, not bandwidth).
__device__ inline double dot_strided(const double* __restrict__ A, size_t lda, const double* __restrict__ x,
                                     int j0, int n, int step) {
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int j = j0;
  for (; j + 7 * step < n; j += 8 * step) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = A[(size_t)(j + u * step) * lda];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += v[u] * x[j + u * step];
  }
  double rest = 0.0;
  for (; j < n; j += step) rest += A[(size_t)j * lda] * x[j];
  return (((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]))) + rest;
}

// Sum of one value per thread, returned to every thread (red: kNT doubles of LDS).
// Sum over the workgroup, identical on every thread: butterfly shuffles inside
// each wave, then the wave sums in wave order (fixed, so bitwise reproducible).
// red needs one double per wave.
__device__ inline double wg_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < nw; ++w) r += red[w];
  __syncthreads();
  return r;
}

// Sum of n partials by every block in the same fixed order.
// Eight loads in flight per thread; the additions keep the plain strided order.
__device__ inline double block_sum_of(const double* __restrict__ v, int n, double* red) {
  double acc = 0.0;
  int i = threadIdx.x;
  for (; i + 7 * kNT < n; i += 8 * kNT) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = v[i + u * kNT];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += t[u];
  }
  for (; i < n; i += kNT) acc += v[i];
  return wg_sum(acc, red);
}

// Lower-triangular solve L y = y in place for a single right-hand side held in
// LDS (y), with L dense in global memory.  Blocked by 16: wave 0 resolves each
// 16 x 16 diagonal block with lane shuffles, then the whole workgroup applies
// the block column to the rows below.
__device__ inline void wg_trsv_lower(const double* L, int ldl, int n, double* y) {
  const int tid = threadIdx.x;
  for (int j0 = 0; j0 < n; j0 += 16) {
    const int jb = min(16, n - j0);
    if (tid < 64) {
      const int lane = tid;
      double yi = (lane < jb) ? y[j0 + lane] : 0.0;
      double row[16];
#pragma unroll
      for (int k = 0; k < 16; ++k)
        row[k] = (lane < jb && k <= lane && k < jb) ? L[(j0 + lane) + (size_t)(j0 + k) * ldl] : 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (k < jb) {
          if (lane == k) yi = yi / row[k];
          const double yk = __shfl(yi, k, 64);
          if (lane > k) yi -= row[k] * yk;
        }
      }
      if (lane < jb) y[j0 + lane] = yi;
    }
    __syncthreads();
    for (int i = j0 + jb + tid; i < n; i += kNT) {
      double acc = 0.0;
      for (int k = 0; k < jb; ++k) acc += L[i + (size_t)(j0 + k) * ldl] * y[j0 + k];
      y[i] -= acc;
    }
    __syncthreads();
  }
}

// Solve L^T x = y in place (single right-hand side in LDS), blocked by 16 from the bottom.
__device__ inline void wg_trsv_lower_trans(const double* L, int ldl, int n, double* y) {
  const int tid = threadIdx.x;
  const int nb = (n + 15) / 16;
  for (int b = nb - 1; b >= 0; --b) {
    const int j0 = b * 16;
    const int jb = min(16, n - j0);
    if (tid < 64) {
      const int lane = tid;
      double xi = (lane < jb) ? y[j0 + lane] : 0.0;
      double col[16];   // col[k] = L(j0+k, j0+lane) = (L^T)(lane, k), k >= lane
#pragma unroll
      for (int k = 0; k < 16; ++k)
        col[k] = (lane < jb && k >= lane && k < jb) ? L[(j0 + k) + (size_t)(j0 + lane) * ldl] : 0.0;
#pragma unroll
      for (int kk = 15; kk >= 0; --kk) {
        if (kk < jb) {
          if (lane == kk) xi = xi / col[kk];
          const double xk = __shfl(xi, kk, 64);
          if (lane < kk) xi -= col[kk] * xk;
        }
      }
      if (lane < jb) y[j0 + lane] = xi;
    }
    __syncthreads();
    for (int i = tid; i < j0; i += kNT) {
      double acc = 0.0;
      for (int k = 0; k < jb; ++k) acc += L[(j0 + k) + (size_t)i * ldl] * y[j0 + k];
      y[i] -= acc;
    }
    __syncthreads();
  }
}

}  // namespace bddc
