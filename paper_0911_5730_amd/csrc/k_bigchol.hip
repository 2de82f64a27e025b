// Interior elimination of large substructures (Section 2: the interior
// correction and the Schur complement onto the interface, Section 5's
// reduction to the interface) with FP64 MFMA, for local matrices far larger
// than LDS: a left-looking blocked Cholesky of the first n_I columns of the
// dense local matrix K_s (column-major, n x n), which leaves L_II (lower),
// L_GI (rows n_I.. of the first n_I columns) and the interface Schur
// complement S = K_GG - L_GI L_GI^T (full) in place, as the panel kernels do.
//
// One workgroup of 8 waves per substructure.  The columns are cut into
// blocks of at most 64 (n_I is a block boundary), rows into tiles on the same
// boundaries.  For column block K and every row tile I at or below it:
//   C = A_IK - sum over interior column blocks J < K of L_IJ L_KJ^T,
// with the two 64 x 64 operand tiles of each J staged in LDS by coalesced
// loads and the 16 output tiles of 16 x 16 accumulated on the matrix cores
// (v_mfma_f64_16x16x4f64, two per wave).  Interior K: the diagonal tile is
// factored in LDS (L_KK) and inverted (W = L_KK^-1); every tile below becomes
// L_IK = C W^T, one more 64 x 64 x 64 product on the matrix cores.  Interface
// K: C is the Schur complement block.  Each entry of the factor is read from
// memory once per later column block (left-looking: no read-modify-write of a
// trailing matrix).
#include "dense.hpp"
#include "kernels.hpp"

namespace bddc {

namespace {

typedef double big_d4 __attribute__((ext_vector_type(4)));

constexpr int kBigNT = 512;   // 8 waves
constexpr int kBT = 64;       // tile size
constexpr int kBLd = 68;      // LDS leading dimension of a tile (padded against bank conflicts)

// column block b: [start, end); interior blocks tile [0, nI), interface blocks [nI, n)
struct Blocks {
  int nI, n, nbI, nb;
  __device__ Blocks(int nI_, int n_) : nI(nI_), n(n_) {
    nbI = (nI + kBT - 1) / kBT;
    nb = nbI + (n - nI + kBT - 1) / kBT;
  }
  __device__ int start(int b) const { return b < nbI ? b * kBT : nI + (b - nbI) * kBT; }
  __device__ int end(int b) const { return b < nbI ? min(nI, (b + 1) * kBT) : min(n, nI + (b - nbI + 1) * kBT); }
};

// rows [r0, r0 + rows) x columns [c0, c0 + w) of A (ld n) into the LDS tile T,
// zero-padded to 64 x 64; eight loads in flight per thread
__device__ inline void stage(double* T, const double* __restrict__ A, int n, int r0, int rows, int c0, int w) {
#pragma unroll
  for (int pass = 0; pass < kBT * kBT / (8 * kBigNT); ++pass) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = threadIdx.x + (pass * 8 + u) * kBigNT;
      const int i = idx & (kBT - 1), j = idx >> 6;
      v[u] = (i < rows && j < w) ? A[(r0 + i) + (size_t)(c0 + j) * n] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = threadIdx.x + (pass * 8 + u) * kBigNT;
      T[(idx & (kBT - 1)) + (idx >> 6) * kBLd] = v[u];
    }
  }
}

// acc[h] += (X Y^T) on the two 16 x 16 output tiles t = wave + 8h of the 64 x
// 64 block (rows 16 (t % 4).., columns 16 (t / 4)..), over the first kw
// (padded to 4) columns of the LDS tiles X and Y.  Operands are swapped so
// that register r of lane l holds output (row 16 (t % 4) + l % 16, column
// 16 (t / 4) + l / 16 + 4 r): sixteen consecutive lanes, sixteen consecutive
// rows of one column.
__device__ inline void mma64(big_d4 (&acc)[2], const double* X, const double* Y, int kw) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kw4 = (kw + 3) & ~3;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = wave + 8 * h;
    const int ri = 16 * (t & 3) + (lane & 15), cj = 16 * (t >> 2) + (lane & 15);
    for (int k = 0; k < kw4; k += 4) {
      const int kk = k + (lane >> 4);
      const double a = Y[cj + kk * kBLd];
      const double b = X[ri + kk * kBLd];
      acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[h], 0, 0, 0);
    }
  }
}

template <class F>
__device__ inline void for_acc(F f) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = wave + 8 * h;
    const int i = 16 * (t & 3) + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) f(h, r, i, 16 * (t >> 2) + (lane >> 4) + 4 * r);
  }
}

}  // namespace

// L.tprof (when set) gives each row tile's first interior column tile with a
// nonzero (the envelope of the local matrix, which the factor keeps): tiles
// left of it are zero and are neither formed nor read.  The inverses of the
// interior diagonal tiles are also written to Wd (64 x 64 each, offsets
// L.woff) for the tiled interior solves.
__global__ void __launch_bounds__(kBigNT) k_partial_chol_big(LevelDev L, double* __restrict__ K,
                                                             double* __restrict__ Wd, int* status) {
  extern __shared__ double lds[];
  double* X = lds;                 // operand tile (row tile I), then C
  double* Y = X + kBT * kBLd;      // operand tile (column block K)
  double* W = Y + kBT * kBLd;      // L_KK, then its inverse
  __shared__ double piv[kBT];
  __shared__ double colk[kBT];
  const int s = L.order ? L.order[blockIdx.x] : blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  double* A = K + L.koff[s];
  const Blocks B(nI, n);
  const int32_t* prof = L.tprof ? L.tprof + L.tproff[s] : nullptr;
  double* Ws = Wd + L.woff[s];
  const int tid = threadIdx.x;
  for (int kb = 0; kb < B.nb; ++kb) {
    const int c0 = B.start(kb), w = B.end(kb) - c0;
    const bool interior = kb < B.nbI;
    const int nJ = min(kb, B.nbI);   // interior column blocks left of K
    const int pk = prof ? prof[kb] : 0;
    for (int ib = kb; ib < B.nb; ++ib) {
      const int r0 = B.start(ib), rows = B.end(ib) - r0;
      const bool diag = ib == kb;
      const int pi = prof ? prof[ib] : 0;
      if (interior && pi > kb) continue;   // L_IK = 0 outside the envelope
      big_d4 acc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
      for (int jb = max(pi, pk); jb < nJ; ++jb) {
        const int j0 = B.start(jb), jw = B.end(jb) - j0;
        __syncthreads();   // the tiles of the previous step are consumed
        stage(X, A, n, r0, rows, j0, jw);
        if (!diag) stage(Y, A, n, c0, w, j0, jw);
        __syncthreads();
        mma64(acc, X, diag ? X : Y, jw);
      }
      __syncthreads();
      // C = A_IK - acc into X (a diagonal tile: its lower triangle)
      for_acc([&](int h, int r, int i, int j) {
        double v = 0.0;
        if (i < rows && j < w && (!diag || i >= j)) v = A[(r0 + i) + (size_t)(c0 + j) * n] - acc[h][r];
        X[i + j * kBLd] = v;
      });
      __syncthreads();
      if (!interior) {
        // interface block: Schur complement entries (lower part; mirrored below)
        for_acc([&](int, int, int i, int j) {
          if (i < rows && j < w && (!diag || i >= j)) A[(r0 + i) + (size_t)(c0 + j) * n] = X[i + j * kBLd];
        });
        continue;
      }
      if (diag) {
        // L_KK by right-looking elimination in LDS, then W = L_KK^-1 by
        // in-place Gauss-Jordan steps on the triangle
        for (int k = 0; k < w; ++k) {
          __syncthreads();   // the previous step's updates are complete
          if (tid == 0) {
            const double d = X[k + k * kBLd];
            const bool ok = d > 0.0 && d < 1e308;
            if (!ok) flag_bad(status);
            piv[0] = ok ? sqrt(d) : 1.0;
          }
          __syncthreads();
          const double sq = piv[0];
          for (int i = k + 1 + tid; i < w; i += kBigNT) X[i + k * kBLd] /= sq;
          __syncthreads();
          if (tid == 0) X[k + k * kBLd] = sq;
          const int m = w - k - 1;
          for (int idx = tid; idx < m * m; idx += kBigNT) {
            const int i = k + 1 + idx % m, j = k + 1 + idx / m;
            if (i >= j) X[i + j * kBLd] -= X[i + k * kBLd] * X[j + k * kBLd];
          }
        }
        __syncthreads();
        for (int idx = tid; idx < kBT * kBT; idx += kBigNT) {
          const int i = idx & (kBT - 1), j = idx >> 6;
          W[i + j * kBLd] = (i < w && j < w && i >= j) ? X[i + j * kBLd] : 0.0;
          if (i < w && j < w && i >= j) A[(r0 + i) + (size_t)(c0 + j) * n] = X[i + j * kBLd];
        }
        __syncthreads();
        for (int k = 0; k < w; ++k) {
          const double d = 1.0 / W[k + k * kBLd];
          if (tid < k) piv[tid] = W[k + tid * kBLd] * d;          // row k left of the pivot, scaled
          if (tid > k && tid < w) colk[tid] = W[tid + k * kBLd];  // column k below the pivot
          __syncthreads();
          if (tid < k) W[k + tid * kBLd] = piv[tid];
          if (tid == 0) W[k + k * kBLd] = d;
          for (int idx = tid; idx < w * (k + 1); idx += kBigNT) {
            const int i = idx % w, c = idx / w;
            if (i > k) W[i + c * kBLd] = (c == k) ? -colk[i] * d : W[i + c * kBLd] - colk[i] * piv[c];
          }
          __syncthreads();
        }
        for (int idx = tid; idx < kBT * kBT; idx += kBigNT)
          Ws[(size_t)kb * kBT * kBT + idx] = W[(idx & (kBT - 1)) + (idx >> 6) * kBLd];
        continue;
      }
      // L_IK = C W^T
      big_d4 out[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
      mma64(out, X, W, w);
      for_acc([&](int h, int r, int i, int j) {
        if (i < rows && j < w) A[(r0 + i) + (size_t)(c0 + j) * n] = out[h][r];
      });
    }
  }
  __syncthreads();
  // the Schur complement full (upper from lower)
  const int ng = n - nI;
  for (ColWalk w_(tid, kBigNT, ng); w_.j < ng; w_.next()) {
    const int i = w_.i, c = w_.j;
    [[maybe_unused]] const int idx = i + c * ng;
    if (i < c) A[(nI + i) + (size_t)(nI + c) * n] = A[(nI + c) + (size_t)(nI + i) * n];
  }
}

size_t partial_chol_big_lds() { return sizeof(double) * 3 * kBT * kBLd; }

void launch_partial_chol_big(hipStream_t st, const LevelDev& L, double* K, double* Wd, int* status) {
  if (L.nsub == 0) return;
  launch_kernel(k_partial_chol_big, dim3(L.nsub), dim3(kBigNT), partial_chol_big_lds(), st, L, K, Wd, status);
}

}  // namespace bddc
