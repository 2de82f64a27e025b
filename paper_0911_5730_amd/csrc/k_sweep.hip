// Level-1 interior sweeps of Algorithm "Multilevel BDDC" streamed through LDS:
// the interior pre-correction (eqs. ML-uIi, ML-rBi), the interior
// post-correction (eqs. ML-vIi, ML-ui) and, in the interface-reduced form, the
// static condensation and the interior recovery.
//
// After the interior elimination each substructure matrix holds the n x n_I
// lower trapezoid [L_II; L_GI] (column-major, ld n).  Both sweeps run over that
// trapezoid in 64-column panels:
//   forward:  w = [r_I; 0]   ->  [L_II^{-1} r_I; -L_GI L_II^{-1} r_I]
//   backward: w = [v; u_B]   ->  [L_II^{-T} (v - L_GI^T u_B); u_B]
// A panel (rows from its first column to n) sits in LDS while one wave solves
// its 64 x 64 diagonal block with shuffles and all threads apply the
// off-diagonal part; the next panel's global loads are issued into registers
// before that work starts, so the stream of L never waits on the sweep's
// dependency chain.
#include <cstdlib>
#include <string>

#include "dense.hpp"
#include "kernels.hpp"

namespace bddc {

namespace {

// Panel width BW = 64 (one workgroup per CU, fewest panels) or 32 (LDS of
// 80 KB, two workgroups per CU: for grids of several rounds of workgroups)
constexpr int kSweepNT = 512;              // 8 waves: the prefetch stays within a wave's 63 outstanding loads
constexpr int kSweepRows = 304;            // largest n handled here (LDS: 8 (304 + 304 * 64) B < 160 KiB)
template <int BW>
constexpr int kRegs = (kSweepRows * BW + kSweepNT - 1) / kSweepNT;   // prefetched doubles per thread
// minimum waves per SIMD the register allocation must allow (32-wide: four,
// i.e. two 8-wave workgroups per CU, at most 128 VGPRs per thread)
template <int BW>
constexpr int kSweepBlocks = BW == 32 ? 4 : 1;

// value of v on lane `lane` (uniform) through the scalar unit
__device__ inline double lane_value(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// A panel holds columns [c0, c1) of the rows that can be nonzero there: the
// interior rows [c0, ri) and the interface rows [nI, n).  ri comes from the
// envelope of the local matrix (the factor keeps it: L[i][j] = 0 left of row
// i's first nonzero), so the interior rows past the band are neither loaded
// nor swept; without an envelope ri = nI (every row below c0).
struct Panel {
  int c0, c1, rows;                        // columns [c0, c1), `rows` panel rows
  int ri, nI;
  __device__ int row(int r) const { return r < ri - c0 ? c0 + r : nI + (r - (ri - c0)); }
  __device__ int local(int i) const { return i < ri ? i - c0 : (ri - c0) + (i - nI); }
};

// panel b of BW columns; rend: the envelope's interior row ends of the
// substructure's panels (null: every row)
template <int BW>
__device__ inline Panel panel_of(int b, int n, int nI, const int32_t* rend) {
  Panel p;
  p.c0 = b * BW;
  p.c1 = min(p.c0 + BW, nI);
  const int nb = (nI + BW - 1) / BW;
  p.ri = (rend && b >= 0 && b < nb) ? max(p.c1, min(nI, (int)rend[b])) : nI;
  p.nI = nI;
  p.rows = (p.ri - p.c0) + (n - nI);
  return p;
}

// the interior row ends of substructure s for BW-wide panels (64-wide panels
// first, then 32-wide), or null
template <int BW>
__device__ inline const int32_t* panel_ends(const LevelDev& L, int s) {
  if (!L.srend) return nullptr;
  const int32_t* e = L.srend + L.srendoff[s];
  return BW == 64 ? e : e + (L.nint[s] + 63) / 64;
}

// issue the loads of panel p (its rows x cols [c0, c1) of A) into registers
template <int BW>
__device__ inline void panel_load(const double* __restrict__ A, int n, const Panel& p, double (&r)[kRegs<BW>]) {
  const int w = p.c1 - p.c0;
  ColWalk cw(threadIdx.x, kSweepNT, p.rows);
#pragma unroll
  for (int u = 0; u < kRegs<BW>; ++u) {
    r[u] = cw.j < w ? A[p.row(cw.i) + (size_t)(p.c0 + cw.j) * n] : 0.0;
    cw.next();
  }
}

// the first global row >= i0 with i0's residue mod 8 that lies in the panel
// (rows between ri and nI are skipped; the stride-8 pattern over global rows
// is the dense sweep's, so every partial sum keeps its terms and order)
__device__ inline int next_row8(const Panel& p, int i) {
  return (i >= p.ri && i < p.nI) ? i + ((p.nI - i + 7) / 8) * 8 : i;
}

// store panel registers into LDS: P[(i - c0) + k * rows]
template <int BW>
__device__ inline void panel_store(double* P, const Panel& p, const double (&r)[kRegs<BW>]) {
  const int tot = p.rows * (p.c1 - p.c0);
#pragma unroll
  for (int u = 0; u < kRegs<BW>; ++u) {
    const int idx = threadIdx.x + u * kSweepNT;
    if (idx < tot) P[idx] = r[u];
  }
}

template <int BW>
__device__ __forceinline__ void sweep_fwd(const double* __restrict__ A, int n, int nI, double* w, double* P,
                                          const int32_t* rend) {
  const int tid = threadIdx.x;
  const int nb = (nI + BW - 1) / BW;
  double r[kRegs<BW>];
  Panel p = panel_of<BW>(0, n, nI, rend);
  panel_load<BW>(A, n, p, r);
  panel_store<BW>(P, p, r);
  __syncthreads();
  for (int b = 0; b < nb; ++b) {
    const Panel q = panel_of<BW>(b + 1, n, nI, rend);
    if (b + 1 < nb) panel_load<BW>(A, n, q, r);
    const int wb = p.c1 - p.c0;
    if (tid < 64) {
      // diagonal block: lane l owns row c0 + l
      const int l = tid;
      double wl = l < wb ? w[p.c0 + l] : 0.0;
      const double inv = l < wb ? 1.0 / P[l + l * p.rows] : 0.0;
      for (int j = 0; j < wb; ++j) {
        const double xj = lane_value(wl * inv, j);
        if (l == j) wl = xj;
        else if (l > j && l < wb) wl -= P[l + j * p.rows] * xj;
      }
      if (l < wb) w[p.c0 + l] = wl;
    }
    __syncthreads();
    // rows below the block
    for (int rr = wb + tid; rr < p.rows; rr += kSweepNT) {
      double acc = 0.0;
      const double* Pi = P + rr;
#pragma unroll 8
      for (int k = 0; k < wb; ++k) acc += Pi[k * p.rows] * w[p.c0 + k];
      w[p.row(rr)] -= acc;
    }
    __syncthreads();
    if (b + 1 < nb) {
      panel_store<BW>(P, q, r);
      __syncthreads();
    }
    p = q;
  }
}

template <int BW>
__device__ __forceinline__ void sweep_bwd(const double* __restrict__ A, int n, int nI, double* w, double* P,
                                          const int32_t* rend) {
  const int tid = threadIdx.x;
  const int nb = (nI + BW - 1) / BW;
  double r[kRegs<BW>];
  Panel p = panel_of<BW>(nb - 1, n, nI, rend);
  panel_load<BW>(A, n, p, r);
  panel_store<BW>(P, p, r);
  __syncthreads();
  for (int b = nb - 1; b >= 0; --b) {
    const Panel q = panel_of<BW>(b - 1, n, nI, rend);
    if (b > 0) panel_load<BW>(A, n, q, r);
    const int wb = p.c1 - p.c0;
    // w_j -= sum over rows below the block of L[i][j] w_i, eight lanes per column
    {
      const int j = tid >> 3, part = tid & 7;
      double acc = 0.0;
      if (j < wb)
        for (int i = next_row8(p, p.c0 + wb + part); i < n; i = next_row8(p, i + 8))
          acc += P[p.local(i) + j * p.rows] * w[i];
      acc += __shfl_xor(acc, 1);
      acc += __shfl_xor(acc, 2);
      acc += __shfl_xor(acc, 4);
      __syncthreads();
      if (j < wb && part == 0) w[p.c0 + j] -= acc;
    }
    __syncthreads();
    if (tid < 64) {
      // diagonal block of L^T, from its last row up: lane l owns row c0 + l
      const int l = tid;
      double wl = l < wb ? w[p.c0 + l] : 0.0;
      const double inv = l < wb ? 1.0 / P[l + l * p.rows] : 0.0;
      for (int j = wb - 1; j >= 0; --j) {
        const double xj = lane_value(wl * inv, j);
        if (l == j) wl = xj;
        else if (l < j) wl -= P[j + l * p.rows] * xj;
      }
      if (l < wb) w[p.c0 + l] = wl;
    }
    __syncthreads();
    if (b > 0) {
      panel_store<BW>(P, q, r);
      __syncthreads();
    }
    p = q;
  }
}

// The same sweeps for R columns of w (column c at w + c kSweepRows), 32-wide
// panels: each panel is read once for all columns; wave c solves column c's
// diagonal block, and every column's arithmetic is that of the one-column
// sweep with 32-wide panels.
constexpr int kCBW = 32;

__device__ __forceinline__ void sweep_fwd_cols(const double* __restrict__ A, int n, int nI, double* w, int R,
                                               double* P, const int32_t* rend) {
  const int tid = threadIdx.x, wave = tid >> 6;
  const int nb = (nI + kCBW - 1) / kCBW;
  double r[kRegs<kCBW>];
  Panel p = panel_of<kCBW>(0, n, nI, rend);
  panel_load<kCBW>(A, n, p, r);
  panel_store<kCBW>(P, p, r);
  __syncthreads();
  for (int b = 0; b < nb; ++b) {
    const Panel q = panel_of<kCBW>(b + 1, n, nI, rend);
    if (b + 1 < nb) panel_load<kCBW>(A, n, q, r);
    const int wb = p.c1 - p.c0;
    if (wave < R) {
      // diagonal block of column `wave`: lane l owns row c0 + l
      double* wc = w + wave * kSweepRows;
      const int l = tid & 63;
      double wl = l < wb ? wc[p.c0 + l] : 0.0;
      const double inv = l < wb ? 1.0 / P[l + l * p.rows] : 0.0;
      for (int j = 0; j < wb; ++j) {
        const double xj = lane_value(wl * inv, j);
        if (l == j) wl = xj;
        else if (l > j && l < wb) wl -= P[l + j * p.rows] * xj;
      }
      if (l < wb) wc[p.c0 + l] = wl;
    }
    __syncthreads();
    // rows below the block, every column
    const int below = p.rows - wb;
    for (int t = tid; t < below * R; t += kSweepNT) {
      const int c = t / below, rr = wb + (t - c * below);
      double* wc = w + c * kSweepRows;
      double acc = 0.0;
      const double* Pi = P + rr;
#pragma unroll 8
      for (int k = 0; k < wb; ++k) acc += Pi[k * p.rows] * wc[p.c0 + k];
      wc[p.row(rr)] -= acc;
    }
    __syncthreads();
    if (b + 1 < nb) {
      panel_store<kCBW>(P, q, r);
      __syncthreads();
    }
    p = q;
  }
}

__device__ __forceinline__ void sweep_bwd_cols(const double* __restrict__ A, int n, int nI, double* w, int R,
                                               double* P, const int32_t* rend) {
  const int tid = threadIdx.x, wave = tid >> 6;
  const int nb = (nI + kCBW - 1) / kCBW;
  double r[kRegs<kCBW>];
  Panel p = panel_of<kCBW>(nb - 1, n, nI, rend);
  panel_load<kCBW>(A, n, p, r);
  panel_store<kCBW>(P, p, r);
  __syncthreads();
  for (int b = nb - 1; b >= 0; --b) {
    const Panel q = panel_of<kCBW>(b - 1, n, nI, rend);
    if (b > 0) panel_load<kCBW>(A, n, q, r);
    const int wb = p.c1 - p.c0;
    // w_j -= sum over rows below the block of L[i][j] w_i, eight lanes per
    // (column, j); the rows read lie below the block, the rows written in it
    for (int base = 0; base < wb * R; base += kSweepNT / 8) {
      const int pr = base + (tid >> 3), part = tid & 7;
      const int c = pr / wb, j = pr - c * wb;
      double acc = 0.0;
      if (pr < wb * R) {
        const double* wc = w + c * kSweepRows;
        for (int i = next_row8(p, p.c0 + wb + part); i < n; i = next_row8(p, i + 8))
          acc += P[p.local(i) + j * p.rows] * wc[i];
      }
      acc += __shfl_xor(acc, 1);
      acc += __shfl_xor(acc, 2);
      acc += __shfl_xor(acc, 4);
      if (pr < wb * R && part == 0) w[c * kSweepRows + p.c0 + j] -= acc;
    }
    __syncthreads();
    if (wave < R) {
      // diagonal block of L^T, from its last row up: lane l owns row c0 + l
      double* wc = w + wave * kSweepRows;
      const int l = tid & 63;
      double wl = l < wb ? wc[p.c0 + l] : 0.0;
      const double inv = l < wb ? 1.0 / P[l + l * p.rows] : 0.0;
      for (int j = wb - 1; j >= 0; --j) {
        const double xj = lane_value(wl * inv, j);
        if (l == j) wl = xj;
        else if (l < j) wl -= P[j + l * p.rows] * xj;
      }
      if (l < wb) wc[p.c0 + l] = wl;
    }
    __syncthreads();
    if (b > 0) {
      panel_store<kCBW>(P, q, r);
      __syncthreads();
    }
    p = q;
  }
}

}  // namespace

// The condensation and the interior recovery of the interface-reduced solve
// for R right-hand sides at once (column c of r, y, t, x, u at c times its
// stride): y = L_II^{-1} r_I, t = L_GI y ...
__global__ void __launch_bounds__(kSweepNT, kSweepBlocks<32>) k_sweep_pre_cols(LevelDev L, const double* __restrict__ r,
                                                                               int64_t ldr, double* __restrict__ y, int ldy,
                                                                               double* __restrict__ t, int ldt, int R) {
  extern __shared__ double sh[];
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  double* w = sh;
  double* P = sh + (size_t)R * kSweepRows;
  const int tid = threadIdx.x;
  for (int q = tid; q < n * R; q += kSweepNT) {
    const int c = q / n, i = q - c * n;
    w[c * kSweepRows + i] = i < nI ? r[(size_t)c * ldr + L.int_gid[L.ioff[s] + i]] : 0.0;
  }
  __syncthreads();
  if (nI > 0) sweep_fwd_cols(L.K + L.koff[s], n, nI, w, R, P, panel_ends<kCBW>(L, s));
  for (int q = tid; q < n * R; q += kSweepNT) {
    const int c = q / n, i = q - c * n;
    if (i < nI) y[(size_t)c * ldy + L.ioff[s] + i] = w[c * kSweepRows + i];
    else t[(size_t)c * ldt + L.goff[s] + i - nI] = -w[c * kSweepRows + i];
  }
}

// ... and u_G = x, u_I = L_II^{-T}(y - L_GI^T x_s)
__global__ void __launch_bounds__(kSweepNT, kSweepBlocks<32>) k_sweep_recover_cols(
    LevelDev L, const double* __restrict__ x, int ldx, const double* __restrict__ y, int ldy, double* __restrict__ u,
    int64_t ldu, int R) {
  extern __shared__ double sh[];
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int g0 = L.goff[s];
  double* w = sh;
  double* P = sh + (size_t)R * kSweepRows;
  const int tid = threadIdx.x;
  for (int q = tid; q < ng * R; q += kSweepNT) {
    const int c = q / ng, a = q - c * ng;
    const int f = g0 + a;
    const int gi = L.gam_iid[f];
    const double v = x[(size_t)c * ldx + gi];
    w[c * kSweepRows + nI + a] = v;
    if (L.sh_flat[L.sh_ptr[gi]] == f) u[(size_t)c * ldu + L.gam_gid[f]] = v;
  }
  for (int q = tid; q < nI * R; q += kSweepNT) {
    const int c = q / nI, i = q - c * nI;
    w[c * kSweepRows + i] = y[(size_t)c * ldy + L.ioff[s] + i];
  }
  __syncthreads();
  if (nI == 0) return;
  sweep_bwd_cols(L.K + L.koff[s], n, nI, w, R, P, panel_ends<kCBW>(L, s));
  for (int q = tid; q < nI * R; q += kSweepNT) {
    const int c = q / nI, i = q - c * nI;
    u[(size_t)c * ldu + L.int_gid[L.ioff[s] + i]] = w[c * kSweepRows + i];
  }
}

// y = L_II^{-1} r_I (kept for the post-correction), t = L_GI y
template <int BW>
__global__ void __launch_bounds__(kSweepNT, kSweepBlocks<BW>) k_sweep_pre(LevelDev L, const double* __restrict__ r) {
  extern __shared__ double sh[];
  if (L.stop && *L.stop) return;
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const double* A = L.K + L.koff[s];
  double* w = sh;
  double* P = sh + kSweepRows;
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += kSweepNT) w[i] = i < nI ? r[L.int_gid[L.ioff[s] + i]] : 0.0;
  __syncthreads();
  if (nI > 0) sweep_fwd<BW>(A, n, nI, w, P, panel_ends<BW>(L, s));
  for (int i = tid; i < nI; i += kSweepNT) L.y[L.ioff[s] + i] = w[i];
  for (int a = tid; a < ng; a += kSweepNT) L.t[L.goff[s] + a] = -w[nI + a];
}

// u_B = sum over sharers of v (owner writes); u_I = L_II^{-T} (y - L_GI^T u_B)
template <int BW>
__global__ void __launch_bounds__(kSweepNT, kSweepBlocks<BW>) k_sweep_post(LevelDev L, double* __restrict__ u,
                                                    const int32_t* __restrict__ gam_map) {
  extern __shared__ double sh[];
  if (L.stop && *L.stop) return;
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int g0 = L.goff[s];
  double* w = sh;
  double* P = sh + kSweepRows;
  const int tid = threadIdx.x;
  for (int a = tid; a < ng; a += kSweepNT) {
    const int f = g0 + a;
    const int gi = L.gam_iid[f];
    double acc = 0.0;
    for (int k = L.sh_ptr[gi]; k < L.sh_ptr[gi + 1]; ++k) acc += L.v[L.sh_flat[k]];
    w[nI + a] = acc;
    if (L.sh_flat[L.sh_ptr[gi]] == f) u[gam_map[f]] = acc;
  }
  for (int i = tid; i < nI; i += kSweepNT) w[i] = L.y[L.ioff[s] + i];
  __syncthreads();
  if (nI == 0) return;
  sweep_bwd<BW>(L.K + L.koff[s], n, nI, w, P, panel_ends<BW>(L, s));
  for (int i = tid; i < nI; i += kSweepNT) u[L.int_gid[L.ioff[s] + i]] = w[i];
}

// interior recovery of the interface-reduced solve: u_G = x, u_I = L_II^{-T}(y - L_GI^T x_s)
template <int BW>
__global__ void __launch_bounds__(kSweepNT, kSweepBlocks<BW>) k_sweep_recover(LevelDev L, const double* __restrict__ x,
                                                       double* __restrict__ u) {
  extern __shared__ double sh[];
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int g0 = L.goff[s];
  double* w = sh;
  double* P = sh + kSweepRows;
  const int tid = threadIdx.x;
  for (int a = tid; a < ng; a += kSweepNT) {
    const int f = g0 + a;
    const int gi = L.gam_iid[f];
    const double v = x[gi];
    w[nI + a] = v;
    if (L.sh_flat[L.sh_ptr[gi]] == f) u[L.gam_gid[f]] = v;
  }
  for (int i = tid; i < nI; i += kSweepNT) w[i] = L.y[L.ioff[s] + i];
  __syncthreads();
  if (nI == 0) return;
  sweep_bwd<BW>(L.K + L.koff[s], n, nI, w, P, panel_ends<BW>(L, s));
  for (int i = tid; i < nI; i += kSweepNT) u[L.int_gid[L.ioff[s] + i]] = w[i];
}

template <int BW>
constexpr size_t sweep_lds_bytes() { return sizeof(double) * ((size_t)kSweepRows + (size_t)kSweepRows * BW); }
static_assert(sweep_lds_bytes<64>() <= 160 * 1024, "sweep LDS");
static_assert(2 * sweep_lds_bytes<32>() <= 160 * 1024, "two 32-wide sweep workgroups per CU");

bool sweep_fits(int nmax) { return nmax <= kSweepRows; }

static size_t sweep_cols_lds(int R) { return sizeof(double) * ((size_t)R * kSweepRows + (size_t)kSweepRows * kCBW); }
static_assert(sizeof(double) * ((size_t)kMaxRhs * kSweepRows + (size_t)kSweepRows * kCBW) <= 160 * 1024,
              "column sweeps of kMaxRhs columns");

void launch_sweep_pre_cols(hipStream_t st, const LevelDev& L, const double* r, int64_t ldr, double* y, int ldy, double* t,
                           int ldt, int R) {
  if (L.nsub == 0 || R == 0) return;
  launch_kernel(k_sweep_pre_cols, dim3(L.nsub), dim3(kSweepNT), sweep_cols_lds(R), st, L, r, ldr, y, ldy, t, ldt, R);
}
void launch_sweep_recover_cols(hipStream_t st, const LevelDev& L, const double* x, int ldx, const double* y, int ldy,
                               double* u, int64_t ldu, int R) {
  if (L.nsub == 0 || R == 0) return;
  launch_kernel(k_sweep_recover_cols, dim3(L.nsub), dim3(kSweepNT), sweep_cols_lds(R), st, L, x, ldx, y, ldy, u, ldu,
                R);
}

// 32-wide panels once the grid takes more than one round of one workgroup per
// CU (BDDC_SWEEP_BW=32/64 forces either width)
static bool narrow_panels(int nsub) {
  const char* env = getenv("BDDC_SWEEP_BW");
  if (env) return std::string(env) == "32";
  return nsub > 256;
}

void launch_sweep_pre(hipStream_t st, const LevelDev& L, const double* r) {
  if (narrow_panels(L.nsub))
    launch_kernel(k_sweep_pre<32>, dim3(L.nsub), dim3(kSweepNT), sweep_lds_bytes<32>(), st, L, r);
  else
    launch_kernel(k_sweep_pre<64>, dim3(L.nsub), dim3(kSweepNT), sweep_lds_bytes<64>(), st, L, r);
}
void launch_sweep_post(hipStream_t st, const LevelDev& L, double* u, const int32_t* gam_map) {
  if (narrow_panels(L.nsub))
    launch_kernel(k_sweep_post<32>, dim3(L.nsub), dim3(kSweepNT), sweep_lds_bytes<32>(), st, L, u, gam_map);
  else
    launch_kernel(k_sweep_post<64>, dim3(L.nsub), dim3(kSweepNT), sweep_lds_bytes<64>(), st, L, u, gam_map);
}
void launch_sweep_recover(hipStream_t st, const LevelDev& L, const double* x, double* u) {
  if (narrow_panels(L.nsub))
    launch_kernel(k_sweep_recover<32>, dim3(L.nsub), dim3(kSweepNT), sweep_lds_bytes<32>(), st, L, x, u);
  else
    launch_kernel(k_sweep_recover<64>, dim3(L.nsub), dim3(kSweepNT), sweep_lds_bytes<64>(), st, L, x, u);
}

}  // namespace bddc
