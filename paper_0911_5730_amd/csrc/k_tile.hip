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
// One workgroup of four waves per substructure.  Every tile product runs on
// the matrix cores: wave w owns rows 16 w .. 16 w + 15 of the 64-row output
// block and all columns, and loads its operands straight from memory into
// registers in the instruction's layout -- no LDS staging of the operator
// tiles and no barrier inside a row tile's sum.  Lane l = 16 q + i' supplies
// the operator entry of row i' and reduction index k = 4 s + q at step s of
// the 16 steps of a 64-wide product: for a tile read as stored (L_IJ, W)
// sixteen consecutive rows of four adjacent columns per load, for a tile read
// transposed (L_GI^T, L_JI^T, W^T) four consecutive rows of sixteen columns.
// Up to four right-hand sides take v_mfma_f64_4x4x4f64 (four 4 x 4 x 4
// blocks: block b rows 4 b .. 4 b + 3 of the wave's sixteen, lane l the
// right-hand-side column l mod 4; results on lane 16 i + 4 b + j: row 4 b + i,
// column j); five to eight take v_mfma_f64_16x16x4f64 (lane l the column
// l mod 16, zero past eight; results on lane 16 q + i': row i', columns q and
// 4 + q).  Both shapes form every entry as the chain of four fused
// multiply-adds in k order (measured bitwise on MI355X), and the steps run in
// the same order, so a column solved alone equals the same column of a
// blocked solve bitwise.  Entries known to be zero are not loaded: those
// left of the envelope (per four rows, the first column of the factor's
// nonzeros) and the upper triangle of W.  They are exact zeros, so the sums
// are the same.
#include "dense.hpp"
#include "kernels.hpp"

namespace bddc {

namespace {

constexpr int kTT = 64;   // tile size
constexpr int kXS = 9;    // LDS row stride of an operand block: entry (k, c) at k kXS + c (c < 8)

static_assert(kMaxRhs == 8, "the tile products hold eight columns");

typedef double tile_d4 __attribute__((ext_vector_type(4)));

// The accumulators of one lane: the 4 x 4 x 4 form one entry (row orow,
// column ocol(0)), the 16 x 16 x 4 form two (columns ocol(0), ocol(1)).
template <bool kWide> struct TileAcc;
template <> struct TileAcc<false> {
  double a = 0.0;
  __device__ double get(int) const { return a; }
};
template <> struct TileAcc<true> {
  tile_d4 a = {0.0, 0.0, 0.0, 0.0};
  __device__ double get(int h) const { return a[h]; }
};

// acc += the tile product over the 64 reduction indices: lane l = 16 q + i'
// holds t[s] = op(T)(i', 4 s + q) and x[s] = X(4 s + q, xcol)
template <bool kWide>
__device__ inline void mma_tile(TileAcc<kWide>& acc, const double (&t)[16], const double (&x)[16]) {
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    if constexpr (kWide) acc.a = __builtin_amdgcn_mfma_f64_16x16x4f64(x[s], t[s], acc.a, 0, 0, 0);
    else acc.a = __builtin_amdgcn_mfma_f64_4x4x4f64(t[s], x[s], acc.a, 0, 0, 0);
  }
}

template <bool kWide>
struct TileLane {
  int li, lq, ib;
  int orow;   // the row (within the tile) of the lane's results
  int xcol;   // the right-hand-side column the lane supplies to the products
  static constexpr int kOut = kWide ? 2 : 1;   // results per lane
  __device__ TileLane() {
    const int lane = threadIdx.x & 63;
    li = lane & 15;
    lq = lane >> 4;
    ib = 16 * __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    orow = kWide ? ib + li : ib + (li & 12) + lq;
    xcol = kWide ? li : (li & 3);
  }
  __device__ int ocol(int h) const { return kWide ? lq + 4 * h : (li & 3); }   // the column of result h
};

}  // namespace

// y = L_II^-1 r_I (columns at ldy, interior flat) and t = L_GI y (at ldt,
// interface flat) for R columns of r (at ldr, level dofs); kWide: R > 4
// (held to 128 registers: four workgroups per compute unit, every
// substructure's workgroup resident at once for 1024 substructures)
template <bool kWide>
__global__ void __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(4)))
k_tile_pre_cols(LevelDev L, const double* __restrict__ r, int64_t ldr, double* __restrict__ yout, int ldy,
                double* __restrict__ tout, int ldt, int R) {
  using Lane = TileLane<kWide>;
  extern __shared__ double sh[];
  if (L.stop && *L.stop) return;
  double* xs = sh;   // the right-hand side of the diagonal product, 64 x kXS
  const int s = L.order ? L.order[blockIdx.x] : blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const double* A = L.K + L.koff[s];
  const int32_t* prof = L.tprof + L.tproff[s];
  const double* Ws = L.Wd + L.woff[s];
  const int i0 = L.ioff[s], g0 = L.goff[s];
  const int nbI = (nI + kTT - 1) / kTT, nbG = (ng + kTT - 1) / kTT;
  const Lane T;
  const int32_t* gf = L.rgf ? L.rgf + L.rgfoff[s] : nullptr;   // envelope per four rows
  const int nI4 = (nI + 3) / 4;
  double* yI = yout + i0;   // column c at yI + c ldy
  for (int I = 0; I < nbI; ++I) {
    const int r0 = I * kTT, rows = min(kTT, nI - r0);
    const int row = r0 + T.ib + T.li;   // the row of the operator entries this lane loads
    const bool row_ok = T.ib + T.li < rows;
    const int fr = !row_ok ? INT32_MAX : gf ? gf[row >> 2] : 0;   // the row's first column to load
    const int orow = r0 + T.orow;       // the row of this lane's results
    const bool orow_ok = T.orow < rows;
    // this lane's entries of f_I (its result row and columns), loaded first
    double f[Lane::kOut];
    {
      const int gid = orow_ok ? L.int_gid[i0 + orow] : 0;
#pragma unroll
      for (int h = 0; h < Lane::kOut; ++h)
        f[h] = (orow_ok && T.ocol(h) < R) ? r[(size_t)T.ocol(h) * ldr + gid] : 0.0;
    }
    TileAcc<kWide> acc;
    for (int J = prof[I]; J < I; ++J) {
      double t[16], x[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int k = J * kTT + 4 * q + T.lq;
        t[q] = k >= fr ? A[row + (size_t)k * n] : 0.0;
        x[q] = T.xcol < R ? yI[(size_t)T.xcol * ldy + k] : 0.0;
      }
      mma_tile<kWide>(acc, t, x);
    }
    // b = f_I - sum L_IJ y_J (rows past the tile and columns past R are zero)
#pragma unroll
    for (int h = 0; h < Lane::kOut; ++h) xs[T.orow * kXS + T.ocol(h)] = f[h] - acc.get(h);
    __syncthreads();
    TileAcc<kWide> y4;
    {
      const double* WI = Ws + (size_t)I * kTT * kTT;
      double t[16], x[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int k = 4 * q + T.lq;
        t[q] = (row_ok && k <= T.ib + T.li) ? WI[(T.ib + T.li) + k * kTT] : 0.0;   // (W lower triangular)
        x[q] = T.xcol < kMaxRhs ? xs[k * kXS + T.xcol] : 0.0;
      }
      mma_tile<kWide>(y4, t, x);
    }
#pragma unroll
    for (int h = 0; h < Lane::kOut; ++h)
      if (orow_ok && T.ocol(h) < R) yI[(size_t)T.ocol(h) * ldy + orow] = y4.get(h);
    __syncthreads();   // xs is rewritten, and y_I is read by the later row tiles
  }
  for (int G = 0; G < nbG; ++G) {
    const int r0 = nI + G * kTT, rows = min(kTT, n - r0);
    const int row = r0 + T.ib + T.li;
    const bool row_ok = T.ib + T.li < rows;
    const int fr = !row_ok ? INT32_MAX : gf ? gf[nI4 + ((G * kTT + T.ib + T.li) >> 2)] : 0;
    TileAcc<kWide> acc;
    for (int J = prof[nbI + G]; J < nbI; ++J) {
      double t[16], x[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int k = J * kTT + 4 * q + T.lq;
        t[q] = (k >= fr && k < nI) ? A[row + (size_t)k * n] : 0.0;
        x[q] = (T.xcol < R && k < nI) ? yI[(size_t)T.xcol * ldy + k] : 0.0;
      }
      mma_tile<kWide>(acc, t, x);
    }
#pragma unroll
    for (int h = 0; h < Lane::kOut; ++h)
      if (T.orow < rows && T.ocol(h) < R) tout[(size_t)T.ocol(h) * ldt + g0 + G * kTT + T.orow] = acc.get(h);
  }
}

// u_G = x (interface values at ldx, interface index; the owner writes u),
// u_I = L_II^-T (y - L_GI^T u_G) for R columns (y at ldy, interior flat; u at
// ldu, level dofs); kWide: R > 4.  y is overwritten: each row tile's entries
// by u_I once that tile is solved (the earlier tiles read u_J there,
// contiguous).
template <bool kWide>
__global__ void __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(4)))
k_tile_recover_cols(LevelDev L, const double* __restrict__ x, int ldx, double* __restrict__ y, int ldy,
                    double* __restrict__ u, int64_t ldu, int R, int ngmax) {
  using Lane = TileLane<kWide>;
  extern __shared__ double sh[];
  double* xs = sh;              // the right-hand side of the diagonal product, 64 x kXS
  double* xg = sh + kTT * kXS;  // u_G, ngp x kXS
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
  (void)ngmax;
  for (int idx = tid; idx < ngp * kMaxRhs; idx += kNT) {
    const int a = idx >> 3, c = idx & 7;
    double v = 0.0;
    if (a < ng && c < R) {
      const int f = g0 + a;
      const int gi = L.gam_iid[f];
      v = x[(size_t)c * ldx + gi];
      if (L.sh_flat[L.sh_ptr[gi]] == f) u[(size_t)c * ldu + L.gam_gid[f]] = v;
    }
    xg[a * kXS + c] = v;
  }
  __syncthreads();
  const Lane T;
  // envelope per four rows: at step q of a tile read transposed the four
  // rows of lane group q share one entry (wave-uniform, clamped to the last
  // group; the rows past it are not loaded anyway)
  const int32_t* gf = L.rgf ? L.rgf + L.rgfoff[s] : nullptr;
  const int nI4 = (nI + 3) / 4, ng4 = (ng + 3) / 4;
  double* yI = y + i0;   // y_I in, u_I out
  for (int I = nbI - 1; I >= 0; --I) {
    const int r0 = I * kTT, rows = min(kTT, nI - r0);
    const int col = r0 + T.ib + T.li;   // the column of the transposed tiles this lane loads
    const bool col_ok = T.ib + T.li < rows;
    const int orow = r0 + T.orow;       // the row of u_I this lane's results belong to
    const bool orow_ok = T.orow < rows;
    const int gid = orow_ok ? L.int_gid[i0 + orow] : 0;
    double f[Lane::kOut];
#pragma unroll
    for (int h = 0; h < Lane::kOut; ++h)
      f[h] = (orow_ok && T.ocol(h) < R) ? yI[(size_t)T.ocol(h) * ldy + orow] : 0.0;
    TileAcc<kWide> acc;
    // L_GI^T u_G over the interface tiles whose envelope reaches tile I
    for (int G = 0; G < nbG; ++G) {
      if (prof[nbI + G] > I) continue;
      const int g_0 = nI + G * kTT, grows = min(kTT, n - g_0);
      double t[16], xv[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int k = 4 * q + T.lq;
        const int fq = gf ? gf[nI4 + min(16 * G + q, ng4 - 1)] : 0;
        t[q] = (col_ok && k < grows && col >= fq) ? A[(g_0 + k) + (size_t)col * n] : 0.0;
        xv[q] = T.xcol < kMaxRhs ? xg[(G * kTT + k) * kXS + T.xcol] : 0.0;
      }
      mma_tile<kWide>(acc, t, xv);
    }
    // L_JI^T u_J over the later interior tiles whose envelope reaches tile I
    for (int J = I + 1; J < nbI; ++J) {
      if (prof[J] > I) continue;
      const int j0 = J * kTT, jrows = min(kTT, nI - j0);
      double t[16], xv[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int k = 4 * q + T.lq;
        const int fq = gf ? gf[min(16 * J + q, nI4 - 1)] : 0;
        t[q] = (col_ok && k < jrows && col >= fq) ? A[(j0 + k) + (size_t)col * n] : 0.0;
        xv[q] = (T.xcol < R && k < jrows) ? yI[(size_t)T.xcol * ldy + j0 + k] : 0.0;
      }
      mma_tile<kWide>(acc, t, xv);
    }
#pragma unroll
    for (int h = 0; h < Lane::kOut; ++h) xs[T.orow * kXS + T.ocol(h)] = f[h] - acc.get(h);
    __syncthreads();
    TileAcc<kWide> u4;
    {
      const double* WI = Ws + (size_t)I * kTT * kTT;
      double t[16], xv[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int k = 4 * q + T.lq;
        t[q] = (col_ok && k >= T.ib + T.li && k < rows) ? WI[k + (T.ib + T.li) * kTT] : 0.0;   // (W^T upper)
        xv[q] = T.xcol < kMaxRhs ? xs[k * kXS + T.xcol] : 0.0;
      }
      mma_tile<kWide>(u4, t, xv);
    }
#pragma unroll
    for (int h = 0; h < Lane::kOut; ++h) {
      if (orow_ok && T.ocol(h) < R) {
        yI[(size_t)T.ocol(h) * ldy + orow] = u4.get(h);
        u[(size_t)T.ocol(h) * ldu + gid] = u4.get(h);
      }
    }
    __syncthreads();   // xs is rewritten, and u_I is read by the earlier row tiles
  }
}

static size_t tile_lds(int ngmax) {
  const size_t ngp = (size_t)((ngmax + kTT - 1) / kTT) * kTT;
  return sizeof(double) * (size_t)kXS * (kTT + ngp);
}

void launch_tile_pre_cols(hipStream_t st, const LevelDev& L, const double* r, int64_t ldr, double* y, int ldy,
                          double* t, int ldt, int R) {
  if (R < 1 || R > kMaxRhs) throw std::invalid_argument("launch_tile_pre_cols: bad column count");
  if (R > 4)
    launch_kernel(k_tile_pre_cols<true>, dim3(L.nsub), dim3(kNT), tile_lds(0), st, L, r, ldr, y, ldy, t, ldt, R);
  else
    launch_kernel(k_tile_pre_cols<false>, dim3(L.nsub), dim3(kNT), tile_lds(0), st, L, r, ldr, y, ldy, t, ldt, R);
}

void launch_tile_recover_cols(hipStream_t st, const LevelDev& L, const double* x, int ldx, double* y, int ldy,
                              double* u, int64_t ldu, int R, int ngmax) {
  if (R < 1 || R > kMaxRhs) throw std::invalid_argument("launch_tile_recover_cols: bad column count");
  if (R > 4)
    launch_kernel(k_tile_recover_cols<true>, dim3(L.nsub), dim3(kNT), tile_lds(ngmax), st, L, x, ldx, y, ldy, u, ldu,
                  R, ngmax);
  else
    launch_kernel(k_tile_recover_cols<false>, dim3(L.nsub), dim3(kNT), tile_lds(ngmax), st, L, x, ldx, y, ldy, u,
                  ldu, R, ngmax);
}

}  // namespace bddc
