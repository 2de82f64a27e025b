// Interior solves of large substructures with the tiled factor, for up to
// eight right-hand sides at once (Section 5: the reduction of level 1 to the
// interface condenses the load, y = L_II^-1 f_I and t = L_GI y, and recovers
// the interior at the end, u_I = L_II^-T (y - L_GI^T u_G)).
//
// The factor is the one k_partial_chol_big leaves in the dense local matrix:
// 64 x 64 tiles, the envelope of each row tile (tiles left of it are zero and
// are skipped) and the explicit inverse W of every interior diagonal tile, so
// that each step of the block substitution is a product, never a sequential
// triangular solve:
//   forward  y_I = W_I (f_I - sum_{J in envelope, J < I} L_IJ y_J)
//   backward u_I = W_I^T (y_I - L_GI^T u_G - sum_{J > I} L_JI^T u_J)
// One workgroup per substructure; every operand tile is staged in LDS with
// coalesced loads and applied to all columns from there.
#include "dense.hpp"
#include "kernels.hpp"

namespace bddc {

namespace {

constexpr int kTT = 64;    // tile size
constexpr int kTL = 65;    // LDS leading dimension of a staged tile

// rows [r0, r0 + rows) x columns [c0, c0 + w) of A (column-major, ld lda) into
// Tl, zero-padded to 64 x 64; sixteen loads per thread, all issued first
__device__ inline void stage_tile(double* Tl, const double* __restrict__ A, int64_t lda, int r0, int rows, int c0,
                                  int w) {
  double v[kTT * kTT / kNT];
#pragma unroll
  for (int u = 0; u < kTT * kTT / kNT; ++u) {
    const int idx = threadIdx.x + u * kNT;
    const int i = idx & (kTT - 1), j = idx >> 6;
    v[u] = (i < rows && j < w) ? A[(r0 + i) + (size_t)(c0 + j) * lda] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kTT * kTT / kNT; ++u) {
    const int idx = threadIdx.x + u * kNT;
    Tl[(idx & (kTT - 1)) + (idx >> 6) * kTL] = v[u];
  }
}

// out(i, c) = sum_k op(T)(i, k) x(k, c) for the 64 rows of a staged tile and
// R columns of x (LDS, ld 64): thread (i, q) sums k in [16 q, 16 q + 16), the
// four quarter sums are added in a fixed order.  acc(i, c) (LDS, ld 64) is
// then updated: acc = sign * out + (add ? acc : 0).  Ends with a barrier.
template <bool kTrans>
__device__ inline void tile_product(const double* Tl, const double* x, int R, double* part, double* acc, double sign,
                                    bool add) {
  const int i = threadIdx.x & (kTT - 1), q = threadIdx.x >> 6;
  double s[kMaxRhs];
#pragma unroll
  for (int c = 0; c < kMaxRhs; ++c) s[c] = 0.0;
#pragma unroll 4
  for (int k = 16 * q; k < 16 * q + 16; ++k) {
    const double t = kTrans ? Tl[k + i * kTL] : Tl[i + k * kTL];
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c)
      if (c < R) s[c] += t * x[k + c * kTT];
  }
#pragma unroll
  for (int c = 0; c < kMaxRhs; ++c)
    if (c < R) part[(q * kMaxRhs + c) * kTT + i] = s[c];
  __syncthreads();
  for (int idx = threadIdx.x; idx < kTT * R; idx += kNT) {
    const int ii = idx & (kTT - 1), c = idx >> 6;
    const double v = (part[c * kTT + ii] + part[(kMaxRhs + c) * kTT + ii]) +
                     (part[(2 * kMaxRhs + c) * kTT + ii] + part[(3 * kMaxRhs + c) * kTT + ii]);
    acc[ii + c * kTT] = (add ? acc[ii + c * kTT] : 0.0) + sign * v;
  }
  __syncthreads();
}

struct TileLds {
  double* Tl;     // 64 x 65 operator tile
  double* xb;     // 64 x 8 input tile
  double* bb;     // 64 x 8 accumulator
  double* part;   // 4 x 8 x 64 quarter sums
  double* xg;     // interface values, ngmax x 8 (recovery)
  __device__ TileLds(double* sh) {
    Tl = sh;
    xb = Tl + kTT * kTL;
    bb = xb + kTT * kMaxRhs;
    part = bb + kTT * kMaxRhs;
    xg = part + 4 * kMaxRhs * kTT;
  }
};

}  // namespace

// y = L_II^-1 r_I (columns at ldy, interior flat) and t = L_GI y (at ldt,
// interface flat) for R columns of r (at ldr, level dofs)
__global__ void __launch_bounds__(kNT) k_tile_pre_cols(LevelDev L, const double* __restrict__ r, int64_t ldr,
                                                       double* __restrict__ yout, int ldy, double* __restrict__ tout,
                                                       int ldt, int R) {
  extern __shared__ double sh[];
  if (L.stop && *L.stop) return;
  const TileLds S(sh);
  const int s = L.order ? L.order[blockIdx.x] : blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const double* A = L.K + L.koff[s];
  const int32_t* prof = L.tprof + L.tproff[s];
  const double* Ws = L.Wd + L.woff[s];
  const int i0 = L.ioff[s], g0 = L.goff[s];
  const int nbI = (nI + kTT - 1) / kTT, nbG = (ng + kTT - 1) / kTT;
  const int tid = threadIdx.x;
  for (int I = 0; I < nbI; ++I) {
    const int r0 = I * kTT, rows = min(kTT, nI - r0);
    for (int idx = tid; idx < kTT * R; idx += kNT) {
      const int i = idx & (kTT - 1), c = idx >> 6;
      S.bb[idx] = i < rows ? r[(size_t)c * ldr + L.int_gid[i0 + r0 + i]] : 0.0;
    }
    for (int J = prof[I]; J < I; ++J) {
      stage_tile(S.Tl, A, n, r0, rows, J * kTT, kTT);
      for (int idx = tid; idx < kTT * R; idx += kNT) {
        const int k = idx & (kTT - 1), c = idx >> 6;
        S.xb[idx] = yout[(size_t)c * ldy + i0 + J * kTT + k];
      }
      __syncthreads();
      tile_product<false>(S.Tl, S.xb, R, S.part, S.bb, -1.0, true);
    }
    stage_tile(S.Tl, Ws + (size_t)I * kTT * kTT, kTT, 0, kTT, 0, kTT);
    __syncthreads();
    tile_product<false>(S.Tl, S.bb, R, S.part, S.xb, 1.0, false);
    for (int idx = tid; idx < kTT * R; idx += kNT) {
      const int i = idx & (kTT - 1), c = idx >> 6;
      if (i < rows) yout[(size_t)c * ldy + i0 + r0 + i] = S.xb[idx];
    }
    __syncthreads();
  }
  for (int G = 0; G < nbG; ++G) {
    const int r0 = nI + G * kTT, rows = min(kTT, n - r0);
    for (int idx = tid; idx < kTT * R; idx += kNT) S.bb[idx] = 0.0;
    for (int J = prof[nbI + G]; J < nbI; ++J) {
      const int w = min(kTT, nI - J * kTT);
      stage_tile(S.Tl, A, n, r0, rows, J * kTT, w);
      for (int idx = tid; idx < kTT * R; idx += kNT) {
        const int k = idx & (kTT - 1), c = idx >> 6;
        S.xb[idx] = k < w ? yout[(size_t)c * ldy + i0 + J * kTT + k] : 0.0;
      }
      __syncthreads();
      tile_product<false>(S.Tl, S.xb, R, S.part, S.bb, 1.0, true);
    }
    for (int idx = tid; idx < kTT * R; idx += kNT) {
      const int i = idx & (kTT - 1), c = idx >> 6;
      if (i < rows) tout[(size_t)c * ldt + g0 + G * kTT + i] = S.bb[idx];
    }
    __syncthreads();
  }
}

// u_G = x (interface values at ldx, interface index; the owner writes u),
// u_I = L_II^-T (y - L_GI^T u_G) for R columns (y at ldy, u at ldu, level dofs)
__global__ void __launch_bounds__(kNT) k_tile_recover_cols(LevelDev L, const double* __restrict__ x, int ldx,
                                                           const double* __restrict__ y, int ldy,
                                                           double* __restrict__ u, int64_t ldu, int R, int ngmax) {
  extern __shared__ double sh[];
  const TileLds S(sh);
  const int s = L.order ? L.order[blockIdx.x] : blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const double* A = L.K + L.koff[s];
  const int32_t* prof = L.tprof + L.tproff[s];
  const double* Ws = L.Wd + L.woff[s];
  const int i0 = L.ioff[s], g0 = L.goff[s];
  const int nbI = (nI + kTT - 1) / kTT, nbG = (ng + kTT - 1) / kTT;
  const int tid = threadIdx.x;
  const int ngp = nbG * kTT;   // (<= ngmax rounded up to the tile)
  for (int idx = tid; idx < ngp * R; idx += kNT) {
    const int c = idx / ngp, a = idx - c * ngp;
    double v = 0.0;
    if (a < ng) {
      const int f = g0 + a;
      const int gi = L.gam_iid[f];
      v = x[(size_t)c * ldx + gi];
      if (L.sh_flat[L.sh_ptr[gi]] == f) u[(size_t)c * ldu + L.gam_gid[f]] = v;
    }
    S.xg[idx] = v;
  }
  (void)ngmax;
  __syncthreads();
  for (int I = nbI - 1; I >= 0; --I) {
    const int r0 = I * kTT, rows = min(kTT, nI - r0);
    for (int idx = tid; idx < kTT * R; idx += kNT) {
      const int i = idx & (kTT - 1), c = idx >> 6;
      S.bb[idx] = i < rows ? y[(size_t)c * ldy + i0 + r0 + i] : 0.0;
    }
    // - L_GI^T u_G over the interface tiles whose envelope reaches tile I
    for (int G = 0; G < nbG; ++G) {
      if (prof[nbI + G] > I) continue;
      const int g_0 = nI + G * kTT, grows = min(kTT, n - g_0);
      stage_tile(S.Tl, A, n, g_0, grows, r0, rows);
      for (int idx = tid; idx < kTT * R; idx += kNT) {
        const int k = idx & (kTT - 1), c = idx >> 6;
        S.xb[idx] = S.xg[c * ngp + G * kTT + k];
      }
      __syncthreads();
      tile_product<true>(S.Tl, S.xb, R, S.part, S.bb, -1.0, true);
    }
    // - L_JI^T u_J over the later interior tiles whose envelope reaches tile I
    for (int J = I + 1; J < nbI; ++J) {
      if (prof[J] > I) continue;
      const int j0 = J * kTT, jrows = min(kTT, nI - j0);
      stage_tile(S.Tl, A, n, j0, jrows, r0, rows);
      for (int idx = tid; idx < kTT * R; idx += kNT) {
        const int k = idx & (kTT - 1), c = idx >> 6;
        S.xb[idx] = k < jrows ? u[(size_t)c * ldu + L.int_gid[i0 + j0 + k]] : 0.0;
      }
      __syncthreads();
      tile_product<true>(S.Tl, S.xb, R, S.part, S.bb, -1.0, true);
    }
    stage_tile(S.Tl, Ws + (size_t)I * kTT * kTT, kTT, 0, kTT, 0, kTT);
    __syncthreads();
    tile_product<true>(S.Tl, S.bb, R, S.part, S.xb, 1.0, false);
    for (int idx = tid; idx < kTT * R; idx += kNT) {
      const int i = idx & (kTT - 1), c = idx >> 6;
      if (i < rows) u[(size_t)c * ldu + L.int_gid[i0 + r0 + i]] = S.xb[idx];
    }
    __syncthreads();
  }
}

static size_t tile_lds(int ngmax) {
  const size_t ngp = (size_t)((ngmax + kTT - 1) / kTT) * kTT;
  return sizeof(double) * ((size_t)kTT * kTL + 2 * (size_t)kTT * kMaxRhs + 4 * (size_t)kMaxRhs * kTT + ngp * kMaxRhs);
}

void launch_tile_pre_cols(hipStream_t st, const LevelDev& L, const double* r, int64_t ldr, double* y, int ldy,
                          double* t, int ldt, int R) {
  if (R < 1 || R > kMaxRhs) throw std::invalid_argument("launch_tile_pre_cols: bad column count");
  launch_kernel(k_tile_pre_cols, dim3(L.nsub), dim3(kNT), tile_lds(0), st, L, r, ldr, y, ldy, t, ldt, R);
}

void launch_tile_recover_cols(hipStream_t st, const LevelDev& L, const double* x, int ldx, const double* y, int ldy,
                              double* u, int64_t ldu, int R, int ngmax) {
  if (R < 1 || R > kMaxRhs) throw std::invalid_argument("launch_tile_recover_cols: bad column count");
  launch_kernel(k_tile_recover_cols, dim3(L.nsub), dim3(kNT), tile_lds(ngmax), st, L, x, ldx, y, ldy, u, ldu, R,
                ngmax);
}

}  // namespace bddc
