// The coarsest problem when it is large (Algorithm "Multilevel BDDC": a direct
// solve at level L).  One workgroup factoring A_L and every workgroup of a
// solve sweeping its triangles does not scale to coarse spaces of thousands of
// dofs, so the set-up forms A_L^-1 instead, with a block Gauss-Jordan sweep of
// many workgroups, and each solve is one product with it that reads A_L^-1
// once for all right-hand sides.
//
// Sweep over pivot blocks K of kGJ rows (A column-major n x n, SPD): with
// P = A_KK^-1 and T = A_{:,K} P,
//   A_ij <- A_ij - T_i A_Kj     (i, j outside K)
//   A_Kj <- P A_Kj,  A_iK <- -T_i,  A_KK <- P
// After the last block A holds A^-1.  Every pivot block is a Schur complement
// of the SPD matrix, hence SPD, so no pivoting is needed; a non-positive pivot
// flags the status word (bit 1) like the factorizations do.  The result is
// symmetrized at the end.
#include "kernels.hpp"

namespace bddc {

namespace {
constexpr int kGJ = 64;          // pivot block and tile edge
constexpr int kPad = kGJ + 1;    // LDS column stride of the B operand
}

// P = A_KK^-1 by scalar Gauss-Jordan in LDS (one workgroup)
__global__ void __launch_bounds__(kNT) k_gj_pivot(const double* __restrict__ A, int n, int k0, int kb,
                                                  double* __restrict__ P, int* status) {
  __shared__ double M[kGJ * kGJ];
  __shared__ double colp[kGJ], rowp[kGJ];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kb * kb; idx += kNT) {
    const int i = idx % kb, j = idx / kb;
    M[i + j * kGJ] = A[(size_t)(k0 + i) + (size_t)(k0 + j) * n];
  }
  __syncthreads();
  bool bad = false;
  for (int p = 0; p < kb; ++p) {
    if (tid < kb) {
      colp[tid] = M[tid + p * kGJ];
      rowp[tid] = M[p + tid * kGJ];
    }
    __syncthreads();
    const double piv = colp[p];
    bad = bad || !(piv > 0.0);
    const double inv = 1.0 / piv;
    for (int idx = tid; idx < kb * kb; idx += kNT) {
      const int i = idx % kb, j = idx / kb;
      double v;
      if (i == p)
        v = j == p ? inv : rowp[j] * inv;
      else if (j == p)
        v = -colp[i] * inv;
      else
        v = M[i + j * kGJ] - colp[i] * (rowp[j] * inv);
      M[i + j * kGJ] = v;
    }
    __syncthreads();
  }
  if (bad && tid == 0) atomicOr(status, 1);
  for (int idx = tid; idx < kb * kb; idx += kNT) {
    const int i = idx % kb, j = idx / kb;
    P[i + j * kGJ] = M[i + j * kGJ];
  }
}

// 64 x kb products C = X Y, X 64 x kb (LDS, stride kGJ), Y kb x 64 (LDS,
// stride kPad); each thread owns rows tx + 16 a and columns ty + 16 b
__device__ inline void gj_tile_product(const double* X, const double* Y, int kb, double (&acc)[4][4]) {
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int q = 0; q < kb; ++q) {
    double x[4], y[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) x[a] = X[tx + 16 * a + q * kGJ];
#pragma unroll
    for (int b = 0; b < 4; ++b) y[b] = Y[q + (ty + 16 * b) * kPad];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
  }
}

// T = A_{:,K} P for the row tiles outside K (grid: row tiles); T is n x kb, column-major
__global__ void __launch_bounds__(kNT) k_gj_T(const double* __restrict__ A, int n, int k0, int kb,
                                              const double* __restrict__ P, double* __restrict__ T) {
  __shared__ double X[kGJ * kGJ];
  __shared__ double Y[kGJ * kPad];
  const int t = blockIdx.x, i0 = t * kGJ;
  if (i0 == k0) return;
  const int rows = min(kGJ, n - i0);
  for (int idx = threadIdx.x; idx < kGJ * kb; idx += kNT) {
    const int r = idx % kGJ, q = idx / kGJ;
    X[r + q * kGJ] = r < rows ? A[(size_t)(i0 + r) + (size_t)(k0 + q) * n] : 0.0;
  }
  for (int idx = threadIdx.x; idx < kb * kGJ; idx += kNT) {
    const int q = idx % kb, c = idx / kb;
    Y[q + c * kPad] = c < kb ? P[q + c * kGJ] : 0.0;
  }
  __syncthreads();
  double acc[4][4];
  gj_tile_product(X, Y, kb, acc);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = tx + 16 * a, c = ty + 16 * b;
      if (r < rows && c < kb) T[(size_t)(i0 + r) + (size_t)c * n] = acc[a][b];
    }
}

// A_ij -= T_i A_Kj for the tiles outside row block K and column block K (grid: tiles x tiles)
__global__ void __launch_bounds__(kNT) k_gj_update(double* __restrict__ A, int n, int k0, int kb,
                                                   const double* __restrict__ T) {
  __shared__ double X[kGJ * kGJ];
  __shared__ double Y[kGJ * kPad];
  const int i0 = blockIdx.x * kGJ, j0 = blockIdx.y * kGJ;
  if (i0 == k0 || j0 == k0) return;
  const int rows = min(kGJ, n - i0), cols = min(kGJ, n - j0);
  for (int idx = threadIdx.x; idx < kGJ * kb; idx += kNT) {
    const int r = idx % kGJ, q = idx / kGJ;
    X[r + q * kGJ] = r < rows ? T[(size_t)(i0 + r) + (size_t)q * n] : 0.0;
  }
  for (int idx = threadIdx.x; idx < kb * kGJ; idx += kNT) {
    const int q = idx % kb, c = idx / kb;
    Y[q + c * kPad] = c < cols ? A[(size_t)(k0 + q) + (size_t)(j0 + c) * n] : 0.0;
  }
  __syncthreads();
  double acc[4][4];
  gj_tile_product(X, Y, kb, acc);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = tx + 16 * a, c = ty + 16 * b;
      if (r < rows && c < cols) A[(size_t)(i0 + r) + (size_t)(j0 + c) * n] -= acc[a][b];
    }
}

// the panels of block K (grid: tiles): A_Kj <- P A_Kj for column tile j,
// A_iK <- -T_i for row tile i, and A_KK <- P in the tile of K itself
__global__ void __launch_bounds__(kNT) k_gj_panels(double* __restrict__ A, int n, int k0, int kb,
                                                   const double* __restrict__ P, const double* __restrict__ T) {
  __shared__ double X[kGJ * kGJ];
  __shared__ double Y[kGJ * kPad];
  const int t0 = blockIdx.x * kGJ;
  const int w = min(kGJ, n - t0);
  if (t0 == k0) {
    for (int idx = threadIdx.x; idx < kb * kb; idx += kNT) {
      const int i = idx % kb, j = idx / kb;
      A[(size_t)(k0 + i) + (size_t)(k0 + j) * n] = P[i + j * kGJ];
    }
    return;
  }
  for (int idx = threadIdx.x; idx < kGJ * kb; idx += kNT) {
    const int r = idx % kGJ, q = idx / kGJ;
    X[r + q * kGJ] = r < kb ? P[r + q * kGJ] : 0.0;
  }
  for (int idx = threadIdx.x; idx < kb * kGJ; idx += kNT) {
    const int q = idx % kb, c = idx / kb;
    Y[q + c * kPad] = c < w ? A[(size_t)(k0 + q) + (size_t)(t0 + c) * n] : 0.0;
  }
  __syncthreads();
  double acc[4][4];
  gj_tile_product(X, Y, kb, acc);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = tx + 16 * a, c = ty + 16 * b;
      if (r < kb && c < w) A[(size_t)(k0 + r) + (size_t)(t0 + c) * n] = acc[a][b];
    }
  for (int idx = threadIdx.x; idx < w * kb; idx += kNT) {
    const int r = idx % w, q = idx / w;
    A[(size_t)(t0 + r) + (size_t)(k0 + q) * n] = -T[(size_t)(t0 + r) + (size_t)q * n];
  }
}

// A <- (A + A^T) / 2, one thread per pair i < j (grid: n*n threads)
__global__ void __launch_bounds__(kNT) k_symmetrize(double* __restrict__ A, int n) {
  const size_t idx = (size_t)blockIdx.x * kNT + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const int i = (int)(idx % n), j = (int)(idx / n);
  if (i >= j) return;
  const double m = 0.5 * (A[(size_t)i + (size_t)j * n] + A[(size_t)j + (size_t)i * n]);
  A[(size_t)i + (size_t)j * n] = m;
  A[(size_t)j + (size_t)i * n] = m;
}

// r[:, c] = sum of the coarse contributions of b[:, c] (k_coarse_gather per column; grid: blocks, columns)
__global__ void __launch_bounds__(kNT) k_coarse_gather_cols(int nc, const int32_t* __restrict__ csh_ptr,
                                                            const int32_t* __restrict__ csh_flat,
                                                            const double* __restrict__ b, int64_t ldb,
                                                            double* __restrict__ r, int64_t ldr,
                                                            const int32_t* stop) {
  if (stop && *stop) return;
  const int k = blockIdx.x * kNT + threadIdx.x;
  if (k >= nc) return;
  const double* bc = b + (size_t)blockIdx.y * ldb;
  double acc = 0.0;
  for (int q = csh_ptr[k]; q < csh_ptr[k + 1]; ++q) acc += bc[csh_flat[q]];
  r[k + (size_t)blockIdx.y * ldr] = acc;
}

// u[:, c] = A^-1 r[:, c] for ncols <= kMaxRhs columns: one wave per row i,
// reading column i of the symmetric A^-1 once for every column; each column's
// sum has the same order whatever ncols is
__global__ void __launch_bounds__(kNT) k_coarse_inv_apply(int n, const double* __restrict__ Ainv,
                                                          const double* __restrict__ r, int64_t ldr,
                                                          double* __restrict__ u, int64_t ldu, int ncols,
                                                          const int32_t* stop) {
  if (stop && *stop) return;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (kNT / 64) + (threadIdx.x >> 6);
  if (i >= n) return;
  const double* col = Ainv + (size_t)i * n;
  double acc[kMaxRhs];
#pragma unroll
  for (int c = 0; c < kMaxRhs; ++c) acc[c] = 0.0;
  for (int j = lane; j < n; j += 64) {
    const double a = col[j];
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c)
      if (c < ncols) acc[c] += a * r[j + (size_t)c * ldr];
  }
#pragma unroll
  for (int c = 0; c < kMaxRhs; ++c) {
    if (c >= ncols) break;
    double v = acc[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) u[i + (size_t)c * ldu] = v;
  }
}

// host launchers -------------------------------------------------------------

void launch_coarsest_inverse(hipStream_t st, int n, double* A, double* P, double* T, int* status) {
  if (n == 0) return;
  const int nt = (n + kGJ - 1) / kGJ;
  for (int K = 0; K < nt; ++K) {
    const int k0 = K * kGJ, kb = std::min(kGJ, n - k0);
    launch_kernel(k_gj_pivot, dim3(1), dim3(kNT), 0, st, A, n, k0, kb, P, status);
    launch_kernel(k_gj_T, dim3(nt), dim3(kNT), 0, st, A, n, k0, kb, P, T);
    launch_kernel(k_gj_update, dim3(nt, nt), dim3(kNT), 0, st, A, n, k0, kb, T);
    launch_kernel(k_gj_panels, dim3(nt), dim3(kNT), 0, st, A, n, k0, kb, P, T);
  }
  const size_t nn = (size_t)n * n;
  launch_kernel(k_symmetrize, dim3((unsigned)((nn + kNT - 1) / kNT)), dim3(kNT), 0, st, A, n);
}

void launch_coarse_gather_cols(hipStream_t st, int nc, const int32_t* csh_ptr, const int32_t* csh_flat,
                               const double* b, int64_t ldb, double* r, int64_t ldr, int ncols, const int32_t* stop) {
  if (nc == 0 || ncols == 0) return;
  launch_kernel(k_coarse_gather_cols, dim3((nc + kNT - 1) / kNT, ncols), dim3(kNT), 0, st, nc, csh_ptr, csh_flat, b,
                ldb, r, ldr, stop);
}

void launch_coarse_inv_apply(hipStream_t st, int n, const double* Ainv, const double* r, int64_t ldr, double* u,
                             int64_t ldu, int ncols, const int32_t* stop) {
  if (n == 0 || ncols == 0) return;
  if (ncols > kMaxRhs) throw std::invalid_argument("launch_coarse_inv_apply: too many columns");
  launch_kernel(k_coarse_inv_apply, dim3((n + kNT / 64 - 1) / (kNT / 64)), dim3(kNT), 0, st, n, Ainv, r, ldr, u,
                ldu, ncols, stop);
}

}  // namespace bddc
