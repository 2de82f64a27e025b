// Preconditioner apply (Algorithm "Multilevel BDDC", Section 2.1) and the PCG
// vector kernels (Section 5).
//
// Per level, one workgroup per substructure:
//   k_apply_pre      interior pre-correction and residual update (ML-uIi, ML-rBi):
//                    y = L_II^{-1} r_I, t = L_GI y  (r_B on the interface = r - sum t)
//   k_apply_restrict g = D R r_B on the interface; substructure correction
//                    a = T_rr g_r (ML-wDi) and coarse right-hand side b = Psi^T g
//   k_coarse_gather  r_{l+1} = sum_s R_cs^T b_s (ML-coarse, ML-ri+1)
//   k_coarsest_solve direct solve at the last level
//   k_apply_prolong  v = D (a + Psi u_{l+1})     (ML-uBi-1 before the sum)
//   k_apply_post     u_B = sum_s R_s^T v_s; interior post-correction and
//                    combination (ML-vIi, ML-ui): u_I = L_II^{-T}(y - L_GI^T u_B)
// Interface sums run over the sharers of each dof in a fixed order: no atomics,
// results are reproducible run to run.
#include "dense.hpp"
#include "kernels.hpp"

namespace bddc {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// y = L_II^{-1} r_I ; t = L_GI y
__global__ void __launch_bounds__(kNT) k_apply_pre(LevelDev L, const double* __restrict__ r) {
  extern __shared__ double sh[];
  if (L.stop && *L.stop) return;
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const double* A = L.K + L.koff[s];
  double* y = sh;
  double* part = sh + nI;
  const int tid = threadIdx.x;
  for (int i = tid; i < nI; i += kNT) y[i] = r[L.int_gid[L.ioff[s] + i]];
  __syncthreads();
  wg_trsv_lower(A, n, nI, y);
  for (int i = tid; i < nI; i += kNT) L.y[L.ioff[s] + i] = y[i];
  if (ng == 0) return;
  const int nch = max(1, kNT / ng);
  for (ColWalk w_(tid, kNT, ng); w_.j < nch; w_.next()) {
    const int a = w_.i, c = w_.j;
    [[maybe_unused]] const int idx = a + c * ng;
    double acc = 0.0;
    for (int j = c; j < nI; j += nch) acc += A[(nI + a) + (size_t)j * n] * y[j];
    part[idx] = acc;
  }
  __syncthreads();
  for (int a = tid; a < ng; a += kNT) {
    double acc = 0.0;
    for (int c = 0; c < nch; ++c) acc += part[a + c * ng];
    L.t[L.goff[s] + a] = acc;
  }
}

// g = delta (r_Gamma - sum t);  a_r = T_rr g_r, a_c = 0;  b = Psi^T g
// kFS: full-space input (subtract the interior pre-correction t); otherwise the
// input is an interface vector with zero interior residual.  Grid
// (substructures, columns): column c reads r + c ldr and L.t + c ldg, writes
// L.a + c ldg and L.b + c ldc.
// kRK > 0: each thread's first kRK entries of T_rr are held in registers,
// loaded before g is gathered (for grids of few workgroups, where the
// launch is one dependent chain; with many workgroups the 48 registers
// would halve the resident waves).  The sums are the same either way.
template <bool kFS, int kRK>
__global__ void __launch_bounds__(kNT) k_apply_restrict(LevelDev L, const double* __restrict__ r,
                                                        const int32_t* __restrict__ gam_map, int ldr, int ldg,
                                                        int ldc) {
  extern __shared__ double sh[];
  const int s = blockIdx.x;
  {
    const size_t col = blockIdx.y;
    r += col * ldr;
    L.t += col * ldg;
    L.a += col * ldg;
    L.b += col * ldc;
  }
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int n_r = L.nr[s];
  const int ncs = L.coff[s + 1] - L.coff[s];
  const int g0 = L.goff[s];
  double* g = sh;
  double* part = sh + ng;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  // The operators' loads go out first (in-bounds clamped addresses; entries
  // past the block unused) and land while g is gathered: thread (ti, tc) of
  // the row-partial products T_rr g_r (rows n_r <= the workgroup: one item
  // per thread) its first kRK entries of row ti (columns tc, tc + nch, ...),
  // and wave w the first two 64-entry chunks of its first column of Psi.
  const double* T = L.T + L.toff[s];
  const int nch = n_r > 0 ? max(1, kNT / n_r) : 1;
  const bool one = n_r > 0 && n_r <= kNT;
  const int ti = one ? tid % n_r : 0, tc = one ? tid / n_r : nch;
  double tv[kRK > 0 ? kRK : 1];
  if (kRK > 0 && one) {
#pragma unroll
    for (int k = 0; k < kRK; ++k) tv[k] = T[ti + (size_t)min(tc + k * nch, n_r - 1) * n_r];
  }
  const double* P = L.Psi + L.psioff[s];
  double pv[2] = {0.0, 0.0};
  if (ng > 0 && ncs > 0) {
    const int k = min(wave, ncs - 1);
#pragma unroll
    for (int q = 0; q < 2; ++q) pv[q] = P[min(lane + 64 * q, ng - 1) + (size_t)k * ng];
  }
  if (L.stop && *L.stop) return;
  for (int a = tid; a < ng; a += kNT) {
    const int f = g0 + a;
    double v = r[gam_map[f]];
    if (kFS) {
      const int gi = L.gam_iid[f];
      for (int k = L.sh_ptr[gi]; k < L.sh_ptr[gi + 1]; ++k) v -= L.t[L.sh_flat[k]];
    }
    g[a] = L.delta[f] * v;
  }
  __syncthreads();
  if (kRK == 0 && one) {
    for (ColWalk w_(tid, kNT, n_r); w_.j < nch; w_.next()) {
      const int i = w_.i, c = w_.j;
      [[maybe_unused]] const int idx = i + c * n_r;
      part[idx] = dot_strided(T + i, n_r, g, c, n_r, nch);
    }
  } else if (one) {
    if (tc < nch) {
      // the sum of dot_strided over the columns tc, tc + nch, ...: eight
      // interleaved partial sums over the full batches of eight, then the
      // rest in order
      const int cnt = (n_r - tc + nch - 1) / nch;
      const int nfull = cnt & ~7;
      double a8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      double rest = 0.0;
#pragma unroll
      for (int e = 0; e < kRK; ++e) {
        if (e < cnt) {
          const double x = g[tc + e * nch];
          if (e < nfull) a8[e & 7] += tv[e] * x;
          else rest += tv[e] * x;
        }
      }
      for (int e0 = kRK; e0 < cnt; e0 += 8) {   // the rest: eight loads in flight
        double t8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t8[u] = T[ti + (size_t)min(tc + (e0 + u) * nch, n_r - 1) * n_r];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + u;
          if (e < cnt) {
            const double x = g[tc + e * nch];
            if (e < nfull) a8[e & 7] += t8[u] * x;
            else rest += t8[u] * x;
          }
        }
      }
      part[ti + tc * n_r] = (((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]))) + rest;
    }
  } else if (n_r > 0) {
    for (int i = tid; i < n_r; i += kNT) part[i] = dot_strided(T + i, n_r, g, 0, n_r, 1);
  }
  // b = Psi^T g, one wave per coarse dof
  for (int k = wave, m = 0; k < ncs; k += kNT / 64, ++m) {
    double acc = 0.0;
    int a = lane;
    if (m == 0) {
#pragma unroll
      for (int q = 0; q < 2; ++q, a += 64)
        if (a < ng) acc += pv[q] * g[a];
    }
    for (; a < ng; a += 64) acc += P[a + (size_t)k * ng] * g[a];
    acc = wave_sum(acc);
    if (lane == 0) L.b[L.coff[s] + k] = acc;
  }
  __syncthreads();
  if (n_r > 0) {
    const int nc = one ? nch : 1;
    for (int i = tid; i < n_r; i += kNT) {
      double acc = 0.0;
      for (int c = 0; c < nc; ++c) acc += part[i + c * n_r];
      L.a[g0 + i] = acc;
    }
  }
  for (int a = n_r + tid; a < ng; a += kNT) L.a[g0 + a] = 0.0;
}

__global__ void k_coarse_gather(int nc, const int32_t* __restrict__ csh_ptr, const int32_t* __restrict__ csh_flat,
                                const double* __restrict__ b, double* __restrict__ rc, const int32_t* stop) {
  if (stop && *stop) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nc) return;
  double acc = 0.0;
  for (int q = csh_ptr[k]; q < csh_ptr[k + 1]; ++q) acc += b[csh_flat[q]];
  rc[k] = acc;
}

__global__ void __launch_bounds__(kNT) k_coarsest_solve(int nc, const double* __restrict__ Lc,
                                                        const double* __restrict__ rc, double* __restrict__ uc,
                                                        const int32_t* stop) {
  extern __shared__ double y[];
  if (stop && *stop) return;
  for (int i = threadIdx.x; i < nc; i += kNT) y[i] = rc[i];
  __syncthreads();
  wg_trsv_lower(Lc, nc, nc, y);
  wg_trsv_lower_trans(Lc, nc, nc, y);
  for (int i = threadIdx.x; i < nc; i += kNT) uc[i] = y[i];
}

// Coarse gather and direct coarsest solve in one launch, one workgroup per
// column c of b / uc (strides ldb / ldu): the arithmetic of k_coarse_gather
// followed by k_coarsest_solve.
__global__ void __launch_bounds__(kNT) k_coarse_direct_cols(int nc, const int32_t* __restrict__ csh_ptr,
                                                            const int32_t* __restrict__ csh_flat,
                                                            const double* __restrict__ b, int ldb,
                                                            const double* __restrict__ Lc, double* __restrict__ uc,
                                                            int ldu, const int32_t* stop) {
  extern __shared__ double y[];
  if (stop && *stop) return;
  const double* bc = b + (size_t)blockIdx.x * ldb;
  for (int k = threadIdx.x; k < nc; k += kNT) {
    double acc = 0.0;
    for (int q = csh_ptr[k]; q < csh_ptr[k + 1]; ++q) acc += bc[csh_flat[q]];
    y[k] = acc;
  }
  __syncthreads();
  wg_trsv_lower(Lc, nc, nc, y);
  wg_trsv_lower_trans(Lc, nc, nc, y);
  double* u = uc + (size_t)blockIdx.x * ldu;
  for (int i = threadIdx.x; i < nc; i += kNT) u[i] = y[i];
}

// v = delta (a + Psi u_c)
__global__ void __launch_bounds__(kNT) k_apply_prolong(LevelDev L, const double* __restrict__ uc) {
  extern __shared__ double sh[];
  if (L.stop && *L.stop) return;
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int ng = n - L.nint[s];
  const int ncs = L.coff[s + 1] - L.coff[s];
  const int g0 = L.goff[s];
  double* ul = sh;
  for (int k = threadIdx.x; k < ncs; k += kNT) ul[k] = uc[L.cid[L.coff[s] + k]];
  __syncthreads();
  const double* P = L.Psi + L.psioff[s];
  for (int a = threadIdx.x; a < ng; a += kNT) {
    double w = L.a[g0 + a];
    w += dot_strided(P + a, ng, ul, 0, ncs, 1);
    L.v[g0 + a] = L.delta[g0 + a] * w;
  }
}

// u_B = sum over sharers of v (owner writes); kFS: interior u_I = L^{-T}(y - L_GI^T u_B)
template <bool kFS>
__global__ void __launch_bounds__(kNT) k_apply_post(LevelDev L, double* __restrict__ u,
                                                    const int32_t* __restrict__ gam_map) {
  extern __shared__ double sh[];
  if (L.stop && *L.stop) return;
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int g0 = L.goff[s];
  double* uB = sh;
  double* yv = sh + ng;
  const int tid = threadIdx.x;
  for (int a = tid; a < ng; a += kNT) {
    const int f = g0 + a;
    const int gi = L.gam_iid[f];
    double acc = 0.0;
    for (int k = L.sh_ptr[gi]; k < L.sh_ptr[gi + 1]; ++k) acc += L.v[L.sh_flat[k]];
    uB[a] = acc;
    if (L.sh_flat[L.sh_ptr[gi]] == f) u[gam_map[f]] = acc;
  }
  if (!kFS || nI == 0) return;
  __syncthreads();
  const double* A = L.K + L.koff[s];
  for (int j = tid; j < nI; j += kNT) {
    double acc = 0.0;
    for (int a = 0; a < ng; ++a) acc += A[(nI + a) + (size_t)j * n] * uB[a];
    yv[j] = L.y[L.ioff[s] + j] - acc;
  }
  __syncthreads();
  wg_trsv_lower_trans(A, n, nI, yv);
  for (int j = tid; j < nI; j += kNT) u[L.int_gid[L.ioff[s] + j]] = yv[j];
}

// Interface operator of the interface-reduced level 1: q_s = S_s p_s (local),
// summed over sharers afterwards.
__global__ void __launch_bounds__(kNT) k_schur_local(LevelDev L, const double* __restrict__ p,
                                                     double* __restrict__ qloc) {
  extern __shared__ double sh[];
  if (L.stop && *L.stop) return;
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int g0 = L.goff[s];
  const double* S = L.K + L.koff[s] + nI + (size_t)nI * n;
  double* pl = sh;
  double* part = sh + ng;
  const int tid = threadIdx.x;
  for (int a = tid; a < ng; a += kNT) pl[a] = p[L.gam_iid[g0 + a]];
  __syncthreads();
  const int nch = max(1, kNT / ng);
  for (ColWalk w_(tid, kNT, ng); w_.j < nch; w_.next()) {
    const int i = w_.i, c = w_.j;
    [[maybe_unused]] const int idx = i + c * ng;
    double acc = 0.0;
    for (int j = c; j < ng; j += nch) acc += S[i + (size_t)j * n] * pl[j];
    part[idx] = acc;
  }
  __syncthreads();
  for (int i = tid; i < ng; i += kNT) {
    double acc = 0.0;
    for (int c = 0; c < nch; ++c) acc += part[i + c * ng];
    qloc[g0 + i] = acc;
  }
}

// ---------------------------------------------------------------------------
// PCG vector kernels on the level-1 interface.  Reductions: each block writes
// one partial (tree in LDS), a single block sums the partials in a fixed order.
// The scalars live in device memory; once `done` is set the update kernels
// leave x, r, p unchanged, so extra queued iterations are harmless.

__device__ inline double block_sum(double v, double* red) { return wg_sum(v, red); }

__global__ void __launch_bounds__(kNT) k_gather_dot(int nif, const int32_t* __restrict__ sh_ptr,
                                                    const int32_t* __restrict__ sh_flat,
                                                    const double* __restrict__ qloc, const double* __restrict__ p,
                                                    double* __restrict__ q, double* __restrict__ partial) {
  __shared__ double red[kNT];
  double acc = 0.0;
  for (int g = blockIdx.x * kNT + threadIdx.x; g < nif; g += gridDim.x * kNT) {
    double v = 0.0;
    for (int k = sh_ptr[g]; k < sh_ptr[g + 1]; ++k) v += qloc[sh_flat[k]];
    q[g] = v;
    acc += v * p[g];
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(kNT) k_dot_partial(int n, const double* __restrict__ a, const double* __restrict__ b,
                                                     double* __restrict__ partial) {
  __shared__ double red[kNT];
  double acc = 0.0;
  for (int i = blockIdx.x * kNT + threadIdx.x; i < n; i += gridDim.x * kNT) acc += a[i] * b[i];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// single block: which = 0 -> pq, alpha = rz / pq ; 1 -> rr and convergence test ;
// 2 -> rz_new, beta = rz_new / rz ; 3 -> rz (first) ; 4 -> bb = ||f||^2 and the
// threshold rtol^2 bb ; 5 -> initial rr and the test before the first iteration
__global__ void __launch_bounds__(kNT) k_scalar(int which, int nblk, const double* __restrict__ partial,
                                                PcgScalars* sc) {
  __shared__ double red[kNT];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kNT) acc += partial[i];
  acc = block_sum(acc, red);
  if (threadIdx.x != 0) return;
  if (which == 4) { sc->bb = acc; sc->thr2 = sc->rtol2 * acc; return; }
  if (which == 3) { sc->rz = acc; return; }
  if (which == 5) { sc->rr = acc; if (acc <= sc->thr2) sc->done = 1; return; }
  if (sc->done) return;
  if (which == 0) {
    sc->pq = acc;
    sc->alpha = sc->rz / acc;
  } else if (which == 1) {
    sc->rr = acc;
    sc->iters += 1;
    sc->alphas[min(sc->iters - 1, kMaxHist - 1)] = sc->alpha;
    if (acc <= sc->thr2) sc->done = 1;
    if (sc->iters >= sc->maxit) sc->done = (sc->done ? 1 : 2);
  } else if (which == 2) {
    sc->beta = acc / sc->rz;
    sc->betas[min(sc->iters - 1, kMaxHist - 1)] = sc->beta;
    sc->rz = acc;
  }
}

__global__ void k_update_xr(int n, const PcgScalars* __restrict__ sc, const double* __restrict__ p,
                            const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r,
                            double* __restrict__ partial) {
  __shared__ double red[kNT];
  const bool active = sc->done == 0;
  const double al = sc->alpha;
  double acc = 0.0;
  for (int i = blockIdx.x * kNT + threadIdx.x; i < n; i += gridDim.x * kNT) {
    double ri = r[i];
    if (active) {
      x[i] += al * p[i];
      ri -= al * q[i];
      r[i] = ri;
    }
    acc += ri * ri;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ void k_update_p(int n, const PcgScalars* __restrict__ sc, const double* __restrict__ z,
                           double* __restrict__ p, int first) {
  if (!first && sc->done) return;
  const double be = first ? 0.0 : sc->beta;
  for (int i = blockIdx.x * kNT + threadIdx.x; i < n; i += gridDim.x * kNT) p[i] = z[i] + be * p[i];
}

// r = f_Gamma - sum_s t_s (condensed right-hand side), x = 0
__global__ void k_condense(int nif, const int32_t* __restrict__ sh_ptr, const int32_t* __restrict__ sh_flat,
                           const int32_t* __restrict__ iface_gid, const double* __restrict__ f,
                           const double* __restrict__ t, double* __restrict__ r, double* __restrict__ x) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nif) return;
  double v = f[iface_gid[g]];
  for (int k = sh_ptr[g]; k < sh_ptr[g + 1]; ++k) v -= t[sh_flat[k]];
  r[g] = v;
  x[g] = 0.0;
}

// interior recovery: u_Gamma = x, u_I = L^{-T}(y - L_GI^T x_s) with y = L^{-1} f_I
__global__ void __launch_bounds__(kNT) k_recover(LevelDev L, const double* __restrict__ x, double* __restrict__ u) {
  extern __shared__ double sh[];
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int g0 = L.goff[s];
  double* uB = sh;
  double* yv = sh + ng;
  const int tid = threadIdx.x;
  for (int a = tid; a < ng; a += kNT) {
    const int f = g0 + a;
    const int gi = L.gam_iid[f];
    const double v = x[gi];
    uB[a] = v;
    if (L.sh_flat[L.sh_ptr[gi]] == f) u[L.gam_gid[f]] = v;
  }
  if (nI == 0) return;
  __syncthreads();
  const double* A = L.K + L.koff[s];
  for (int j = tid; j < nI; j += kNT) {
    double acc = 0.0;
    for (int a = 0; a < ng; ++a) acc += A[(nI + a) + (size_t)j * n] * uB[a];
    yv[j] = L.y[L.ioff[s] + j] - acc;
  }
  __syncthreads();
  wg_trsv_lower_trans(A, n, nI, yv);
  for (int j = tid; j < nI; j += kNT) u[L.int_gid[L.ioff[s] + j]] = yv[j];
}

// ---------------------------------------------------------------------------
// R right-hand sides at once (R <= kMaxRhs), for substructures too large for
// the column sweeps: every factor entry is read once for all columns, and
// each column's arithmetic is that of the single-column kernels above
// (wg_trsv_lower / wg_trsv_lower_trans and the same sums in the same order).
// Y holds column c at Y + c ldy (LDS).

// L Y = Y: the 16 x 16 diagonal block by a group of 16 lanes per column
// (four columns per wave), the rows below by one thread per row
__device__ inline void wg_trsm_lower_cols(const double* Lm, int ldl, int n, double* Y, int ldy, int R) {
  const int tid = threadIdx.x, lane = tid & 63, q = lane & 15;
  const int c = (tid >> 6) * 4 + (lane >> 4);
  for (int j0 = 0; j0 < n; j0 += 16) {
    const int jb = min(16, n - j0);
    if (c < R) {
      double yi = q < jb ? Y[c * ldy + j0 + q] : 0.0;
      double row[16];
#pragma unroll
      for (int k = 0; k < 16; ++k)
        row[k] = (q < jb && k <= q && k < jb) ? Lm[(j0 + q) + (size_t)(j0 + k) * ldl] : 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (k < jb) {
          if (q == k) yi = yi / row[k];
          const double yk = __shfl(yi, (lane & ~15) + k, 64);
          if (q > k) yi -= row[k] * yk;
        }
      }
      if (q < jb) Y[c * ldy + j0 + q] = yi;
    }
    __syncthreads();
    for (int i = j0 + jb + tid; i < n; i += kNT) {
      double l[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) l[k] = k < jb ? Lm[i + (size_t)(j0 + k) * ldl] : 0.0;
      for (int cc = 0; cc < R; ++cc) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (k < jb) acc += l[k] * Y[cc * ldy + j0 + k];
        Y[cc * ldy + i] -= acc;
      }
    }
    __syncthreads();
  }
}

// L^T X = Y in place, blocked by 16 from the bottom
__device__ inline void wg_trsm_lower_trans_cols(const double* Lm, int ldl, int n, double* Y, int ldy, int R) {
  const int tid = threadIdx.x, lane = tid & 63, q = lane & 15;
  const int c = (tid >> 6) * 4 + (lane >> 4);
  for (int b = (n + 15) / 16 - 1; b >= 0; --b) {
    const int j0 = b * 16;
    const int jb = min(16, n - j0);
    if (c < R) {
      double xi = q < jb ? Y[c * ldy + j0 + q] : 0.0;
      double col[16];
#pragma unroll
      for (int k = 0; k < 16; ++k)
        col[k] = (q < jb && k >= q && k < jb) ? Lm[(j0 + k) + (size_t)(j0 + q) * ldl] : 0.0;
#pragma unroll
      for (int kk = 15; kk >= 0; --kk) {
        if (kk < jb) {
          if (q == kk) xi = xi / col[kk];
          const double xk = __shfl(xi, (lane & ~15) + kk, 64);
          if (q < kk) xi -= col[kk] * xk;
        }
      }
      if (q < jb) Y[c * ldy + j0 + q] = xi;
    }
    __syncthreads();
    for (int i = tid; i < j0; i += kNT) {
      double l[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) l[k] = k < jb ? Lm[(j0 + k) + (size_t)i * ldl] : 0.0;
      for (int cc = 0; cc < R; ++cc) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (k < jb) acc += l[k] * Y[cc * ldy + j0 + k];
        Y[cc * ldy + i] -= acc;
      }
    }
    __syncthreads();
  }
}

// k_apply_pre for R columns: y[:, c] = L_II^-1 r_I[:, c], t[:, c] = L_GI y[:, c]
// (r at stride ldr, y interior flat at ldy, t interface flat at ldt)
__global__ void __launch_bounds__(kNT) k_apply_pre_cols(LevelDev L, const double* __restrict__ r, int64_t ldr,
                                                        double* __restrict__ yout, int ldy, double* __restrict__ tout,
                                                        int ldt, int R) {
  extern __shared__ double sh[];
  if (L.stop && *L.stop) return;
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const double* A = L.K + L.koff[s];
  const int tid = threadIdx.x;
  double* Y = sh;
  double* part = sh + (size_t)R * nI;
  const int i0 = L.ioff[s], g0 = L.goff[s];
  for (int idx = tid; idx < R * nI; idx += kNT) {
    const int c = idx / nI, i = idx - c * nI;
    Y[idx] = r[(size_t)c * ldr + L.int_gid[i0 + i]];
  }
  __syncthreads();
  wg_trsm_lower_cols(A, n, nI, Y, nI, R);
  for (int idx = tid; idx < R * nI; idx += kNT) {
    const int c = idx / nI, i = idx - c * nI;
    yout[(size_t)c * ldy + i0 + i] = Y[idx];
  }
  if (ng == 0) return;
  const int nch = max(1, kNT / ng);
  const int pw = ng * nch;
  for (ColWalk w_(tid, kNT, ng); w_.j < nch; w_.next()) {
    const int a = w_.i, ch = w_.j;
    double acc[kMaxRhs];
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c) acc[c] = 0.0;
    for (int j = ch; j < nI; j += nch) {
      const double l = A[(nI + a) + (size_t)j * n];
#pragma unroll
      for (int c = 0; c < kMaxRhs; ++c)
        if (c < R) acc[c] += l * Y[c * nI + j];
    }
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c)
      if (c < R) part[c * pw + a + ch * ng] = acc[c];
  }
  __syncthreads();
  for (int idx = tid; idx < R * ng; idx += kNT) {
    const int c = idx / ng, a = idx - c * ng;
    double acc = 0.0;
    for (int ch = 0; ch < nch; ++ch) acc += part[c * pw + a + ch * ng];
    tout[(size_t)c * ldt + g0 + a] = acc;
  }
}

// k_recover for R columns: u_B[:, c] = x[:, c] (at ldx), u_I[:, c] =
// L_II^-T (y[:, c] - L_GI^T u_B[:, c]) (y at ldy, u at ldu)
__global__ void __launch_bounds__(kNT) k_recover_cols(LevelDev L, const double* __restrict__ x, int ldx,
                                                      const double* __restrict__ y, int ldy, double* __restrict__ u,
                                                      int64_t ldu, int R) {
  extern __shared__ double sh[];
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int g0 = L.goff[s], i0 = L.ioff[s];
  const int tid = threadIdx.x;
  double* UB = sh;
  double* YV = sh + (size_t)R * ng;
  for (int idx = tid; idx < R * ng; idx += kNT) {
    const int c = idx / ng, a = idx - c * ng;
    const int f = g0 + a;
    const int gi = L.gam_iid[f];
    const double v = x[(size_t)c * ldx + gi];
    UB[idx] = v;
    if (L.sh_flat[L.sh_ptr[gi]] == f) u[(size_t)c * ldu + L.gam_gid[f]] = v;
  }
  if (nI == 0) return;
  __syncthreads();
  const double* A = L.K + L.koff[s];
  for (int j = tid; j < nI; j += kNT) {
    double acc[kMaxRhs];
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c) acc[c] = 0.0;
    for (int a = 0; a < ng; ++a) {
      const double l = A[(nI + a) + (size_t)j * n];
#pragma unroll
      for (int c = 0; c < kMaxRhs; ++c)
        if (c < R) acc[c] += l * UB[c * ng + a];
    }
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c)
      if (c < R) YV[c * nI + j] = y[(size_t)c * ldy + i0 + j] - acc[c];
  }
  __syncthreads();
  wg_trsm_lower_trans_cols(A, n, nI, YV, nI, R);
  for (int idx = tid; idx < R * nI; idx += kNT) {
    const int c = idx / nI, j = idx - c * nI;
    u[(size_t)c * ldu + L.int_gid[i0 + j]] = YV[idx];
  }
}

__global__ void k_copy(int n, const double* __restrict__ a, double* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// ---------------------------------------------------------------------------
static inline int blocks_for(int n) { return n <= 0 ? 1 : (n + kNT - 1) / kNT; }

void launch_apply_pre(hipStream_t st, const LevelDev& L, int nImax, int ngmax, const double* r) {
  const size_t lds = sizeof(double) * ((size_t)nImax + kNT + ngmax);
  launch_kernel(k_apply_pre, dim3(L.nsub), dim3(kNT), lds, st, L, r);
}
void launch_apply_restrict(hipStream_t st, const LevelDev& L, int ngmax, const double* r,
                           const int32_t* gam_map, int use_t) {
  const size_t lds = sizeof(double) * ((size_t)ngmax + kNT + ngmax);
  if (use_t)
    launch_kernel(k_apply_restrict<true, 0>, dim3(L.nsub), dim3(kNT), lds, st, L, r, gam_map, 0, 0, 0);
  else
    launch_kernel(k_apply_restrict<false, 0>, dim3(L.nsub), dim3(kNT), lds, st, L, r, gam_map, 0, 0, 0);
}
void launch_wide_restrict(hipStream_t st, const WideDev& W, const int32_t* gam_map) {
  LevelDev L = W.L;
  L.stop = W.stop;
  const size_t lds = sizeof(double) * ((size_t)W.ngmax + kNT + W.ngmax);
  launch_kernel(k_apply_restrict<true, 24>, dim3(L.nsub, W.nrhs), dim3(kNT), lds, st, L, W.r2, gam_map, W.ld_r2,
                W.ld_g, W.ld_c);
}
void launch_coarse_gather(hipStream_t st, int nc, const int32_t* csh_ptr, const int32_t* csh_flat,
                          const double* b, double* rc, const int32_t* stop) {
  if (nc == 0) return;
  launch_kernel(k_coarse_gather, dim3(blocks_for(nc)), dim3(kNT), 0, st, nc, csh_ptr, csh_flat, b, rc,
                     stop);
}
void launch_coarsest_solve(hipStream_t st, int nc, const double* Lc, const double* rc, double* uc,
                           const int32_t* stop) {
  if (nc == 0) return;
  launch_kernel(k_coarsest_solve, dim3(1), dim3(kNT), sizeof(double) * (size_t)nc, st, nc, Lc, rc, uc,
                     stop);
}
void launch_coarse_direct_cols(hipStream_t st, int nc, const int32_t* csh_ptr, const int32_t* csh_flat,
                               const double* b, int ldb, const double* Lc, double* uc, int ldu, int ncols,
                               const int32_t* stop) {
  if (nc == 0 || ncols == 0) return;
  launch_kernel(k_coarse_direct_cols, dim3(ncols), dim3(kNT), sizeof(double) * (size_t)nc, st, nc, csh_ptr, csh_flat,
                b, ldb, Lc, uc, ldu, stop);
}
void launch_apply_prolong(hipStream_t st, const LevelDev& L, int ncsmax, const double* uc) {
  launch_kernel(k_apply_prolong, dim3(L.nsub), dim3(kNT), sizeof(double) * (size_t)(ncsmax + 1), st, L, uc);
}
void launch_apply_post(hipStream_t st, const LevelDev& L, int nImax, int ngmax, double* u,
                       const int32_t* gam_map, int interior) {
  const size_t lds = sizeof(double) * ((size_t)ngmax + nImax + 1);
  if (interior)
    launch_kernel(k_apply_post<true>, dim3(L.nsub), dim3(kNT), lds, st, L, u, gam_map);
  else
    launch_kernel(k_apply_post<false>, dim3(L.nsub), dim3(kNT), lds, st, L, u, gam_map);
}
void launch_schur_local(hipStream_t st, const LevelDev& L, int ngmax, const double* p, double* qloc) {
  const size_t lds = sizeof(double) * ((size_t)ngmax + kNT + ngmax);
  launch_kernel(k_schur_local, dim3(L.nsub), dim3(kNT), lds, st, L, p, qloc);
}
void launch_gather_dot(hipStream_t st, int nblk, int nif, const int32_t* sh_ptr, const int32_t* sh_flat,
                       const double* qloc, const double* p, double* q, double* partial) {
  launch_kernel(k_gather_dot, dim3(nblk), dim3(kNT), 0, st, nif, sh_ptr, sh_flat, qloc, p, q, partial);
}
void launch_dot_partial(hipStream_t st, int nblk, int n, const double* a, const double* b, double* partial) {
  launch_kernel(k_dot_partial, dim3(nblk), dim3(kNT), 0, st, n, a, b, partial);
}
void launch_scalar(hipStream_t st, int which, int nblk, const double* partial, PcgScalars* sc) {
  launch_kernel(k_scalar, dim3(1), dim3(kNT), 0, st, which, nblk, partial, sc);
}
void launch_update_xr(hipStream_t st, int nblk, int n, const PcgScalars* sc, const double* p, const double* q,
                      double* x, double* r, double* partial) {
  launch_kernel(k_update_xr, dim3(nblk), dim3(kNT), 0, st, n, sc, p, q, x, r, partial);
}
void launch_update_p(hipStream_t st, int nblk, int n, const PcgScalars* sc, const double* z, double* p, int first) {
  launch_kernel(k_update_p, dim3(nblk), dim3(kNT), 0, st, n, sc, z, p, first);
}
void launch_condense(hipStream_t st, int nif, const int32_t* sh_ptr, const int32_t* sh_flat,
                     const int32_t* iface_gid, const double* f, const double* t, double* r, double* x) {
  if (nif == 0) return;
  launch_kernel(k_condense, dim3(blocks_for(nif)), dim3(kNT), 0, st, nif, sh_ptr, sh_flat, iface_gid, f, t,
                     r, x);
}
void launch_recover(hipStream_t st, const LevelDev& L, int nImax, int ngmax, const double* x, double* u) {
  const size_t lds = sizeof(double) * ((size_t)ngmax + nImax + 1);
  launch_kernel(k_recover, dim3(L.nsub), dim3(kNT), lds, st, L, x, u);
}
size_t apply_cols_lds(int R, int nImax, int ngmax) {
  return sizeof(double) * (size_t)R * ((size_t)nImax + (size_t)max(kNT, ngmax));
}
void launch_apply_pre_cols(hipStream_t st, const LevelDev& L, int nImax, int ngmax, const double* r, int64_t ldr,
                           double* y, int ldy, double* t, int ldt, int R) {
  if (L.nsub == 0 || R == 0) return;
  if (R > kMaxRhs) throw std::invalid_argument("launch_apply_pre_cols: too many columns");
  launch_kernel(k_apply_pre_cols, dim3(L.nsub), dim3(kNT), apply_cols_lds(R, nImax, ngmax), st, L, r, ldr, y, ldy, t,
                ldt, R);
}
void launch_recover_cols(hipStream_t st, const LevelDev& L, int nImax, int ngmax, const double* x, int ldx,
                         const double* y, int ldy, double* u, int64_t ldu, int R) {
  if (L.nsub == 0 || R == 0) return;
  if (R > kMaxRhs) throw std::invalid_argument("launch_recover_cols: too many columns");
  launch_kernel(k_recover_cols, dim3(L.nsub), dim3(kNT), apply_cols_lds(R, nImax, ngmax), st, L, x, ldx, y, ldy, u,
                ldu, R);
}
void launch_copy(hipStream_t st, int n, const double* a, double* b) {
  if (n == 0) return;
  launch_kernel(k_copy, dim3(blocks_for(n)), dim3(kNT), 0, st, n, a, b);
}

}  // namespace bddc
