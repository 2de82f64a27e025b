// Fused kernels of the PCG iteration (Section 5) and of the deep levels of
// Algorithm "Multilevel BDDC" (Section 2.1).
//
// * k_deep: every level >= 2 and the coarsest direct solve in ONE workgroup
//   of 16 waves.  Wave w owns the level substructures s = w, w+16, ...; all
//   interior corrections are products with the explicit inverse of the
//   interior Cholesky factor, so each step is a wave-wide matrix-vector
//   product; phases that read other substructures' data are separated by
//   workgroup barriers.  The coarsest Cholesky factor is staged in LDS and
//   solved by one wave.  Used when the deep levels are small.
// * k_pcg_*: one PCG iteration on the level-1 interface in five launches plus
//   the apply.  Scalars (alpha, beta, convergence) are recomputed by every
//   block from the per-block partial sums of the previous launch, in a fixed
//   order, so no scalar-only launches are needed and results stay bitwise
//   reproducible.
#include "dense.hpp"
#include "kernels.hpp"

namespace bddc {

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- wave helpers
// y = Linv r_I ; t = L_GI y   (eqs. ML-uIi, ML-rBi)
__device__ void wv_pre(const LevelDev& L, int s, const double* __restrict__ r, double* ws, int lane) {
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const double* A = L.K + L.koff[s];
  const double* Li = L.Linv + L.linvoff[s];
  double* rI = ws;
  double* y = ws + nI;
  for (int i = lane; i < nI; i += 64) rI[i] = r[L.int_gid[L.ioff[s] + i]];
  wave_sync();
  for (int i = lane; i < nI; i += 64) {
    const double acc = dot_strided(Li + i, nI, rI, 0, i + 1, 1);
    y[i] = acc;
    L.y[L.ioff[s] + i] = acc;
  }
  wave_sync();
  for (int a = lane; a < ng; a += 64) L.t[L.goff[s] + a] = dot_strided(A + nI + a, n, y, 0, nI, 1);
  wave_sync();
}

// g = delta (r_G - sum t) ; a = T_rr g_r (ML-wDi) ; b = Psi^T g (ML-coarse)
__device__ void wv_restrict(const LevelDev& L, int s, const double* __restrict__ r, double* ws, int lane) {
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int ng = n - L.nint[s];
  const int n_r = L.nr[s];
  const int ncs = L.coff[s + 1] - L.coff[s];
  const int g0 = L.goff[s];
  double* g = ws;
  for (int a = lane; a < ng; a += 64) {
    const int f = g0 + a;
    double v = r[L.gam_gid[f]];
    const int gi = L.gam_iid[f];
    for (int k = L.sh_ptr[gi]; k < L.sh_ptr[gi + 1]; ++k) v -= L.t[L.sh_flat[k]];
    g[a] = L.delta[f] * v;
  }
  wave_sync();
  const double* T = L.T + L.toff[s];
  for (int i = lane; i < n_r; i += 64) L.a[g0 + i] = dot_strided(T + i, n_r, g, 0, n_r, 1);
  for (int a = n_r + lane; a < ng; a += 64) L.a[g0 + a] = 0.0;
  const double* P = L.Psi + L.psioff[s];
  for (int k = lane; k < ncs; k += 64) L.b[L.coff[s] + k] = dot_strided(P + (size_t)k * ng, 1, g, 0, ng, 1);
  wave_sync();
}

// v = delta (a + Psi u_c)   (ML-uBi-1 before the sum)
__device__ void wv_prolong(const LevelDev& L, int s, const double* __restrict__ uc, double* ws, int lane) {
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int ng = n - L.nint[s];
  const int ncs = L.coff[s + 1] - L.coff[s];
  const int g0 = L.goff[s];
  double* ul = ws;
  for (int k = lane; k < ncs; k += 64) ul[k] = uc[L.cid[L.coff[s] + k]];
  wave_sync();
  const double* P = L.Psi + L.psioff[s];
  for (int a = lane; a < ng; a += 64) {
    const double w = L.a[g0 + a] + dot_strided(P + a, ng, ul, 0, ncs, 1);
    L.v[g0 + a] = L.delta[g0 + a] * w;
  }
  wave_sync();
}

// u_B = sum over sharers of v (owner writes); u_I = Linv^T (y - L_GI^T u_B)  (ML-vIi, ML-ui)
__device__ void wv_post(const LevelDev& L, int s, double* __restrict__ u, double* ws, int lane) {
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int g0 = L.goff[s];
  double* uB = ws;
  double* yv = ws + ng;
  for (int a = lane; a < ng; a += 64) {
    const int f = g0 + a;
    const int gi = L.gam_iid[f];
    double acc = 0.0;
    for (int k = L.sh_ptr[gi]; k < L.sh_ptr[gi + 1]; ++k) acc += L.v[L.sh_flat[k]];
    uB[a] = acc;
    if (L.sh_flat[L.sh_ptr[gi]] == f) u[L.gam_gid[f]] = acc;
  }
  wave_sync();
  if (nI == 0) return;
  const double* A = L.K + L.koff[s];
  for (int j = lane; j < nI; j += 64)
    yv[j] = L.y[L.ioff[s] + j] - dot_strided(A + nI + (size_t)j * n, 1, uB, 0, ng, 1);
  wave_sync();
  const double* Li = L.Linv + L.linvoff[s];
  for (int i = lane; i < nI; i += 64)
    u[L.int_gid[L.ioff[s] + i]] = dot_strided(Li + (size_t)i * nI, 1, yv, i, nI, 1);
  wave_sync();
}

// ---------------------------------------------------------------- deep levels
__global__ void __launch_bounds__(kDeepNT) k_deep(DeepArgs A) {
  extern __shared__ double sh[];
  if (A.stop && *A.stop) return;
  constexpr int NW = kDeepNT / 64;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double* ws = sh + (size_t)wave * A.wstride;
  for (int k = tid; k < A.n2; k += kDeepNT) {
    double acc = 0.0;
    for (int q = A.csh_ptr1[k]; q < A.csh_ptr1[k + 1]; ++q) acc += A.b1[A.csh_flat1[q]];
    A.rvec[0][k] = acc;
  }
  __syncthreads();
  for (int l = 0; l < A.nlev; ++l) {
    const LevelDev& L = A.lv[l];
    for (int s = wave; s < L.nsub; s += NW) wv_pre(L, s, A.rvec[l], ws, lane);
    __syncthreads();
    for (int s = wave; s < L.nsub; s += NW) wv_restrict(L, s, A.rvec[l], ws, lane);
    __syncthreads();
    double* rn = (l + 1 < A.nlev) ? A.rvec[l + 1] : A.rc_last;
    for (int k = tid; k < L.nc; k += kDeepNT) {
      double acc = 0.0;
      for (int q = L.csh_ptr[k]; q < L.csh_ptr[k + 1]; ++q) acc += L.b[L.csh_flat[q]];
      rn[k] = acc;
    }
    __syncthreads();
  }
  // coarsest level: Cholesky factor staged in LDS, two sweeps by wave 0
  const int nc = A.ncL;
  double* Lc = sh + (size_t)NW * A.wstride;
  double* yc = Lc + (size_t)nc * nc;
  for (int idx = tid; idx < nc * nc; idx += kDeepNT) Lc[idx] = A.LL[idx];
  for (int i = tid; i < nc; i += kDeepNT) yc[i] = A.rc_last[i];
  __syncthreads();
  if (wave == 0) {
    for (int j = 0; j < nc; ++j) {
      const double yj = yc[j] / Lc[j + (size_t)j * nc];
      wave_sync();
      if (lane == 0) yc[j] = yj;
      for (int i = j + 1 + lane; i < nc; i += 64) yc[i] -= Lc[i + (size_t)j * nc] * yj;
      wave_sync();
    }
    for (int j = nc - 1; j >= 0; --j) {
      const double xj = yc[j] / Lc[j + (size_t)j * nc];
      wave_sync();
      if (lane == 0) yc[j] = xj;
      for (int i = lane; i < j; i += 64) yc[i] -= Lc[j + (size_t)i * nc] * xj;
      wave_sync();
    }
  }
  __syncthreads();
  for (int i = tid; i < nc; i += kDeepNT) A.uc_last[i] = yc[i];
  __syncthreads();
  for (int l = A.nlev - 1; l >= 0; --l) {
    const LevelDev& L = A.lv[l];
    const double* uc = (l + 1 < A.nlev) ? A.uvec[l + 1] : A.uc_last;
    for (int s = wave; s < L.nsub; s += NW) wv_prolong(L, s, uc, ws, lane);
    __syncthreads();
    for (int s = wave; s < L.nsub; s += NW) wv_post(L, s, A.uvec[l], ws, lane);
    __syncthreads();
  }
}

size_t deep_lds(int wstride, int ncL) {
  return sizeof(double) * ((size_t)(kDeepNT / 64) * wstride + (size_t)ncL * ncL + ncL + 1);
}

void launch_deep(hipStream_t st, const DeepArgs& A) {
  launch_kernel(k_deep, dim3(1), dim3(kDeepNT), deep_lds(A.wstride, A.ncL), st, A);
}

// ---------------------------------------------------------------- deep levels, one workgroup per substructure
// (used when the deep levels are too large for one workgroup)
__global__ void __launch_bounds__(kNT) k_apply_pre_inv(LevelDev L, const double* __restrict__ r) {
  extern __shared__ double sh[];
  if (L.stop && *L.stop) return;
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const double* A = L.K + L.koff[s];
  const double* Li = L.Linv + L.linvoff[s];
  double* rI = sh;
  double* y = sh + nI;
  double* part = y + nI;
  const int tid = threadIdx.x;
  for (int i = tid; i < nI; i += kNT) rI[i] = r[L.int_gid[L.ioff[s] + i]];
  __syncthreads();
  for (int i = tid; i < nI; i += kNT) {
    const double acc = dot_strided(Li + i, nI, rI, 0, i + 1, 1);
    y[i] = acc;
    L.y[L.ioff[s] + i] = acc;
  }
  __syncthreads();
  if (ng == 0) return;
  const int nch = max(1, kNT / ng);
  for (ColWalk w_(tid, kNT, ng); w_.j < nch; w_.next()) {
    const int a = w_.i, c = w_.j;
    [[maybe_unused]] const int idx = a + c * ng;
    part[idx] = dot_strided(A + nI + a, n, y, c, nI, nch);
  }
  __syncthreads();
  for (int a = tid; a < ng; a += kNT) {
    double acc = 0.0;
    for (int c = 0; c < nch; ++c) acc += part[a + c * ng];
    L.t[L.goff[s] + a] = acc;
  }
}

__global__ void __launch_bounds__(kNT) k_apply_post_inv(LevelDev L, double* __restrict__ u) {
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
    if (L.sh_flat[L.sh_ptr[gi]] == f) u[L.gam_gid[f]] = acc;
  }
  if (nI == 0) return;
  __syncthreads();
  const double* A = L.K + L.koff[s];
  for (int j = tid; j < nI; j += kNT)
    yv[j] = L.y[L.ioff[s] + j] - dot_strided(A + nI + (size_t)j * n, 1, uB, 0, ng, 1);
  __syncthreads();
  const double* Li = L.Linv + L.linvoff[s];
  for (int i = tid; i < nI; i += kNT) u[L.int_gid[L.ioff[s] + i]] = dot_strided(Li + (size_t)i * nI, 1, yv, i, nI, 1);
}

void launch_apply_pre_inv(hipStream_t st, const LevelDev& L, int nImax, int ngmax, const double* r) {
  const size_t lds = sizeof(double) * (2 * (size_t)nImax + kNT + ngmax + 1);
  launch_kernel(k_apply_pre_inv, dim3(L.nsub), dim3(kNT), lds, st, L, r);
}

void launch_apply_post_inv(hipStream_t st, const LevelDev& L, int nImax, int ngmax, double* u) {
  const size_t lds = sizeof(double) * ((size_t)ngmax + nImax + 1);
  launch_kernel(k_apply_post_inv, dim3(L.nsub), dim3(kNT), lds, st, L, u);
}

// ---------------------------------------------------------------- fused PCG iteration
// Sum of n partials by every block in the same fixed order.
__device__ inline double block_sum_of(const double* __restrict__ v, int n, double* red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kNT) acc += v[i];
  return wg_sum(acc, red);
}

// PCG iteration k on the level-1 interface (Section 5) in four launches:
//   matvec   p_k = z + beta p_{k-1};  q_s = S_s p_s;  partial p_s^T q_s
//   update   alpha = rz / p^T S p;  r_k = r_{k-1} - alpha sum_s q_s (every sharer
//            forms the same value, the owner stores it and x += alpha p);
//            partial r.r;  then the restriction of r_k: g = delta r, b = Psi^T g,
//            and delta T_rr g_r published for the interface average
//   deep     levels >= 2 and the coarsest solve
//   average  convergence test on r.r, then z = sum over the sharers s of
//            delta_s (T_rr g_s + Psi_s u_c) and the partial r.z, per interface dof
// p^T S p is summed as the local energies p_s^T S_s p_s, so the assembled q is
// never formed; r is double-buffered by iteration parity because sharers read
// r_{k-1} while owners write r_k.  The average uses, per interface dof, the
// sharers' rows of the delta-weighted coarse basis (built at setup), so the
// prolongation needs no pass of its own.
__global__ void __launch_bounds__(kNT) k_pcg_matvec(LevelDev L, PcgDev P, int it) {
  extern __shared__ double sh[];
  __shared__ double red[kNT];
  if (P.sc->done) return;
  double beta = 0.0;
  if (it >= 2) {
    const double rz = block_sum_of(P.rz_part[(it - 1) & 1], P.nblk, red);
    const double rz0 = block_sum_of(P.rz_part[(it - 2) & 1], P.nblk, red);
    beta = rz / rz0;
    if (blockIdx.x == 0 && threadIdx.x == 0) P.sc->betas[min(it - 2, kMaxHist - 1)] = beta;
  }
  const double* pold = P.p[(it - 1) & 1];
  double* pnew = P.p[it & 1];
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int g0 = L.goff[s];
  const double* S = L.K + L.koff[s] + nI + (size_t)nI * n;
  double* pl = sh;
  double* part = sh + ng;
  const int tid = threadIdx.x;
  for (int a = tid; a < ng; a += kNT) {
    const int f = g0 + a;
    const int gi = L.gam_iid[f];
    const double pv = (it >= 2) ? P.z[gi] + beta * pold[gi] : P.z[gi];
    pl[a] = pv;
    if (L.sh_flat[L.sh_ptr[gi]] == f) pnew[gi] = pv;
  }
  __syncthreads();
  const int nch = max(1, kNT / max(1, ng));
  for (ColWalk w_(tid, kNT, ng); w_.j < nch; w_.next()) {
    const int i = w_.i, c = w_.j;
    [[maybe_unused]] const int idx = i + c * ng;
    part[idx] = dot_strided(S + i, n, pl, c, ng, nch);
  }
  __syncthreads();
  double e = 0.0;
  for (int i = tid; i < ng; i += kNT) {
    double acc = 0.0;
    for (int c = 0; c < nch; ++c) acc += part[i + c * ng];
    P.qloc[g0 + i] = acc;
    e += pl[i] * acc;
  }
  e = wg_sum(e, red);
  if (tid == 0) P.pq_part[s] = e;
}

// Copy n doubles from global src to LDS dst: the first kPre per thread are
// loaded into registers by fetch() (issued early, before other work), the
// rest by finish(), which also stores everything.
template <int kPre>
struct Prefetch {
  double v[kPre];
  const double* src;
  double* dst;
  int n;
  __device__ void fetch(const double* s, double* d, int count) {
    src = s;
    dst = d;
    n = count;
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int i = threadIdx.x + u * kNT;
      v[u] = i < n ? src[i] : 0.0;
    }
  }
  __device__ void finish() {
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int i = threadIdx.x + u * kNT;
      if (i < n) dst[i] = v[u];
    }
    for (int i = threadIdx.x + kPre * kNT; i < n; i += kNT) dst[i] = src[i];
  }
};

// The level-1 restriction of the interface residual r: g = delta r_G,
// b = Psi^T g (ML-coarse) and da = delta T_rr g_r (ML-wDi, weighted for the
// average); g, T_rr (Tl) and Psi (Pl) are already in LDS.
__device__ void pcg_restrict_body(const LevelDev& L, int s, const double* g, double* part, double* da,
                                  const double* T, const double* Pp) {
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int ng = n - L.nint[s];
  const int n_r = L.nr[s];
  const int ncs = L.coff[s + 1] - L.coff[s];
  const int g0 = L.goff[s];
  const int tid = threadIdx.x;
  const int nch = max(1, kNT / max(1, n_r));
  for (ColWalk w_(tid, kNT, n_r); w_.j < nch; w_.next()) {
    const int i = w_.i, c = w_.j;
    [[maybe_unused]] const int idx = i + c * n_r;
    double acc = 0.0;
    for (int k = c; k < n_r; k += nch) acc += T[i + k * n_r] * g[k];
    part[idx] = acc;
  }
  const int wave = tid >> 6, lane = tid & 63;
  for (int k = wave; k < ncs; k += kNT / 64) {
    double acc = 0.0;
    for (int a = lane; a < ng; a += 64) acc += Pp[a + (size_t)k * ng] * g[a];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if (lane == 0) L.b[L.coff[s] + k] = acc;
  }
  __syncthreads();
  for (int i = tid; i < n_r; i += kNT) {
    double acc = 0.0;
    for (int c = 0; c < nch; ++c) acc += part[i + c * n_r];
    da[g0 + i] = L.delta[g0 + i] * acc;
  }
  for (int a = n_r + tid; a < ng; a += kNT) da[g0 + a] = 0.0;
}

// it >= 1: alpha, the residual update (r_k into r[it & 1]) and x update by the
// owners, the partial r.r; then the restriction of r_k.  it == 0: the
// restriction of r_0 only.
__global__ void __launch_bounds__(kNT) k_pcg_update_restrict(LevelDev L, PcgDev P, int it, int nrmax, int ngmax) {
  extern __shared__ double sh[];
  __shared__ double red[kNT];
  if (P.sc->done) return;
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int ng = n - L.nint[s];
  const int g0 = L.goff[s];
  const int tid = threadIdx.x;
  const int n_r = L.nr[s];
  const int ncs = L.coff[s + 1] - L.coff[s];
  double* g = sh;
  double* part = sh + ngmax;
  double* Tl = part + kNT + ngmax;
  double* Pl = Tl + (size_t)nrmax * nrmax;
  // the operators' loads go out first and land while the scalars are formed
  Prefetch<16> pt;
  Prefetch<4> pp;
  pt.fetch(L.T + L.toff[s], Tl, n_r * n_r);
  pp.fetch(L.Psi + L.psioff[s], Pl, ng * ncs);
  if (it == 0) {
    for (int a = tid; a < ng; a += kNT) g[a] = L.delta[g0 + a] * P.r[0][L.gam_iid[g0 + a]];
  } else {
    const double rz = block_sum_of(P.rz_part[(it - 1) & 1], P.nblk, red);
    const double pq = block_sum_of(P.pq_part, P.nsub1, red);
    const double alpha = rz / pq;
    const double* rold = P.r[(it - 1) & 1];
    double* rnew = P.r[it & 1];
    const double* p = P.p[it & 1];
    double rr = 0.0;
    for (int a = tid; a < ng; a += kNT) {
      const int f = g0 + a;
      const int gi = L.gam_iid[f];
      double q = 0.0;
      for (int k = L.sh_ptr[gi]; k < L.sh_ptr[gi + 1]; ++k) q += P.qloc[L.sh_flat[k]];
      const double ri = rold[gi] - alpha * q;
      g[a] = L.delta[f] * ri;
      if (L.sh_flat[L.sh_ptr[gi]] == f) {
        rnew[gi] = ri;
        P.x[gi] += alpha * p[gi];
        rr += ri * ri;
      }
    }
    rr = wg_sum(rr, red);
    if (tid == 0) P.rr_part[s] = rr;
    if (s == 0 && tid == 0) {
      P.sc->iters = it;
      P.sc->alphas[min(it - 1, kMaxHist - 1)] = alpha;
    }
  }
  pt.finish();
  pp.finish();
  __syncthreads();
  pcg_restrict_body(L, s, g, part, P.da, Tl, Pl);
}

// Convergence test on r.r (every block takes the same decision; block 0
// records it), then per interface dof z = sum over sharers of delta T_rr g plus
// the dof's row of the delta-weighted coarse basis times u_c  (ML-uBi-1), and
// the per-block partial of r_k . z.
__global__ void __launch_bounds__(kNT) k_pcg_prolong_post(LevelDev L, PcgDev P, const double* __restrict__ uc,
                                                          int check, int parity) {
  __shared__ double red[kNT];
  if (P.sc->done) return;
  if (check) {
    const double rr = block_sum_of(P.rr_part, P.nsub1, red);
    const bool conv = rr <= P.sc->thr2;
    const bool maxed = P.sc->iters >= P.sc->maxit;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      P.sc->rr = rr;
      if (conv || maxed) P.sc->done = conv ? 1 : 2;
    }
    if (conv || maxed) return;
  }
  // eight lanes per interface dof, fixed-order reduction over the eight
  const double* r = P.r[parity];
  const int gi = (blockIdx.x * kNT + threadIdx.x) >> 3;
  const int sub = threadIdx.x & 7;
  double acc = 0.0;
  if (gi < P.nif) {
    const int k0 = L.sh_ptr[gi], k1 = L.sh_ptr[gi + 1];
    for (int k = k0 + sub; k < k1; k += 8) acc += P.da[L.sh_flat[k]];
    for (int j = P.phi_ptr[gi] + sub; j < P.phi_ptr[gi + 1]; j += 8) acc += P.phi_w[j] * uc[P.phi_ids[j]];
  }
  acc += __shfl_xor(acc, 1);
  acc += __shfl_xor(acc, 2);
  acc += __shfl_xor(acc, 4);
  double rz = 0.0;
  if (gi < P.nif && sub == 0) {
    P.z[gi] = acc;
    rz = acc * r[gi];
  }
  rz = wg_sum(rz, red);
  if (threadIdx.x == 0) P.rz_part[parity][blockIdx.x] = rz;
}

// Rows of the averaged coarse basis: for interface dof gi, in sharer order,
// the coarse ids and delta_s(gi) Psi_s(row of gi, :) of every sharer s.
__global__ void __launch_bounds__(kNT) k_build_phi(LevelDev L, int nif, const int32_t* __restrict__ sub_of_flat,
                                                   const int32_t* __restrict__ phi_ptr, int32_t* __restrict__ phi_ids,
                                                   double* __restrict__ phi_w) {
  const int gi = blockIdx.x * kNT + threadIdx.x;
  if (gi >= nif) return;
  int j = phi_ptr[gi];
  for (int q = L.sh_ptr[gi]; q < L.sh_ptr[gi + 1]; ++q) {
    const int f = L.sh_flat[q];
    const int t = sub_of_flat[f];
    const int at = f - L.goff[t];
    const int ngt = (L.loc_ptr[t + 1] - L.loc_ptr[t]) - L.nint[t];
    const int ncst = L.coff[t + 1] - L.coff[t];
    const double* Pt = L.Psi + L.psioff[t];
    for (int k = 0; k < ncst; ++k) {
      phi_ids[j] = L.cid[L.coff[t] + k];
      phi_w[j++] = L.delta[f] * Pt[at + (size_t)k * ngt];
    }
  }
}

void launch_pcg_matvec(hipStream_t st, const LevelDev& L, int ngmax, const PcgDev& P, int it) {
  const size_t lds = sizeof(double) * ((size_t)ngmax + kNT + ngmax);
  launch_kernel(k_pcg_matvec, dim3(L.nsub), dim3(kNT), lds, st, L, P, it);
}
void launch_pcg_update_restrict(hipStream_t st, const LevelDev& L, int ngmax, int nrmax, int ncsmax, const PcgDev& P,
                                int it) {
  const size_t lds = sizeof(double) * ((size_t)ngmax + kNT + ngmax + (size_t)nrmax * nrmax + (size_t)ngmax * ncsmax);
  launch_kernel(k_pcg_update_restrict, dim3(L.nsub), dim3(kNT), lds, st, L, P, it, nrmax, ngmax);
}
void launch_pcg_prolong_post(hipStream_t st, const LevelDev& L, const PcgDev& P, const double* uc, int check,
                            int parity) {
  launch_kernel(k_pcg_prolong_post, dim3(P.nblk), dim3(kNT), 0, st, L, P, uc, check, parity);
}
void launch_build_phi(hipStream_t st, const LevelDev& L, int nif, const int32_t* sub_of_flat, const int32_t* phi_ptr,
                      int32_t* phi_ids, double* phi_w) {
  if (nif == 0) return;
  launch_kernel(k_build_phi, dim3((nif + kNT - 1) / kNT), dim3(kNT), 0, st, L, nif, sub_of_flat, phi_ptr, phi_ids,
                phi_w);
}

}  // namespace bddc
