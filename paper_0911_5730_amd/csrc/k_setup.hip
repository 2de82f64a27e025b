// Setup kernels: local assembly, stiffness-scaling weights, interior
// elimination (partial Cholesky -> interior factor and interface Schur
// complement), constraint matrices, constrained local factors with the
// energy-minimal coarse basis, and the coarsest-level factor.
//
// One workgroup per substructure; every matrix is dense FP64, column-major,
// with the substructure's local dofs ordered [interior | interface
// non-corner | corner].
#include <algorithm>
#include <cstdlib>
#include <string>

#include "dense.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace bddc {

// ---------------------------------------------------------------------------
// Level-1 assembly (Section 2: a(u,v) = sum_e k_e int grad u . grad v):
// K_s = sum over the elements of s of k_e * Khat.  Thread a owns row a, so the
// accumulation order is fixed and no atomics are needed.  The interface part
// of the diagonal is kept for the stiffness-scaling weights.
// kM element dofs (4 nodes, or 8: two components per node), kBits bits of
// element position in the node_el codes
template <int kM, int kBits, class KH>
__global__ void __launch_bounds__(kNT) k_assemble_l1(
    const int64_t* __restrict__ koff, const int32_t* __restrict__ loc_ptr,
    const int32_t* __restrict__ nint, const int32_t* __restrict__ node_el,
    const int32_t* __restrict__ sub_el_ptr, const int32_t* __restrict__ el_gid,
    const int32_t* __restrict__ el_loc, const double* __restrict__ coeff, KH khat,
    double* __restrict__ K, double* __restrict__ diagK, const int32_t* __restrict__ goff, int* status) {
  const int s = blockIdx.x;
  const int base = loc_ptr[s];
  const int n = loc_ptr[s + 1] - base;
  const int e0 = sub_el_ptr[s];
  double* A = K + koff[s];
  for (int idx = threadIdx.x; idx < n * n; idx += kNT) A[idx] = 0.0;
  __syncthreads();
  for (int a = threadIdx.x; a < n; a += kNT) {
    for (int k = 0; k < 4; ++k) {
      const int code = node_el[(size_t)(base + a) * 4 + k];
      if (code < 0) continue;
      const int le = code >> kBits, pos = code & ((1 << kBits) - 1);
      const double kk = coeff[el_gid[e0 + le]];
      if (!(kk > 0.0 && kk < 1e308)) atomicOr(status, 2);   // check of device-resident input
#pragma unroll
      for (int q = 0; q < kM; ++q) {
        const int b = el_loc[(size_t)(e0 + le) * kM + q];
        if (b >= 0) A[a + (size_t)b * n] += kk * khat.v[pos * kM + q];
      }
    }
    if (a >= nint[s]) diagK[goff[s] + a - nint[s]] = A[a + (size_t)a * n];
  }
}

// Level >= 2 assembly (Section 2.1: level-l elements are level-(l-1)
// substructures with the coarse element matrices A_c as element matrices).
// Children are added one after another, so the sum order is fixed.
__global__ void __launch_bounds__(kNT) k_assemble_coarse(
    const int64_t* __restrict__ koff, const int32_t* __restrict__ loc_ptr,
    const int32_t* __restrict__ nint, const int32_t* __restrict__ child_ptr,
    const int32_t* __restrict__ child_id, const int32_t* __restrict__ child_map_off,
    const int32_t* __restrict__ child_map, const double* __restrict__ Ac,
    const int64_t* __restrict__ acoff, const int32_t* __restrict__ nc_child, double* __restrict__ K,
    double* __restrict__ diagK, const int32_t* __restrict__ goff) {
  const int s = blockIdx.x;
  const int n = loc_ptr[s + 1] - loc_ptr[s];
  double* A = K + koff[s];
  for (int idx = threadIdx.x; idx < n * n; idx += kNT) A[idx] = 0.0;
  __syncthreads();
  for (int slot = child_ptr[s]; slot < child_ptr[s + 1]; ++slot) {
    const int c = child_id[slot];
    const int m = nc_child[c];
    const double* Ae = Ac + acoff[c];
    const int32_t* map = child_map + child_map_off[slot];
    for (ColWalk w_(threadIdx.x, kNT, m); w_.j < m; w_.next()) {
      const int i = w_.i, j = w_.j;
      [[maybe_unused]] const int idx = i + j * m;
      A[map[i] + (size_t)map[j] * n] += Ae[idx];
    }
    __syncthreads();
  }
  for (int a = nint[s] + threadIdx.x; a < n; a += kNT) diagK[goff[s] + a - nint[s]] = A[a + (size_t)a * n];
}

// Stiffness scaling: delta_s(x) = K_s(x,x) / sum_{j in N_x} K_j(x,x) on the
// interface (summed over the sharers of x in a fixed order).
__global__ void k_weights(int nflat, const int32_t* __restrict__ flat_iid,
                          const int32_t* __restrict__ sh_ptr, const int32_t* __restrict__ sh_flat,
                          const double* __restrict__ diagK, double* __restrict__ delta) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nflat) return;
  const int g = flat_iid[f];
  double sum = 0.0;
  for (int k = sh_ptr[g]; k < sh_ptr[g + 1]; ++k) sum += diagK[sh_flat[k]];
  delta[f] = diagK[f] / sum;
}

// ---------------------------------------------------------------------------
// Interior elimination, blocked right-looking Cholesky on the first nI columns
// of K_s.  A panel of kPanel columns is factored in LDS, written back, and used
// for the rank-kPanel update of the trailing lower triangle in 4x4 register
// tiles.  On exit: L_II (lower), L_GI = K_GI L_II^{-T} below it, and the
// interface Schur complement S = K_GG - L_GI L_GI^T, mirrored to full storage.
constexpr int kPanel = 16;

__global__ void __launch_bounds__(kNT) k_partial_chol(const int64_t* __restrict__ koff,
                                                      const int32_t* __restrict__ loc_ptr,
                                                      const int32_t* __restrict__ nint,
                                                      double* __restrict__ K, int* status) {
  extern __shared__ double P[];
  const int s = blockIdx.x;
  const int n = loc_ptr[s + 1] - loc_ptr[s];
  const int nI = nint[s];
  double* A = K + koff[s];
  const int tid = threadIdx.x;
  for (int k0 = 0; k0 < nI; k0 += kPanel) {
    const int kb = min(kPanel, nI - k0);
    const int m = n - k0;
    for (ColWalk w_(tid, kNT, m); w_.j < kb; w_.next()) {
      const int i = w_.i, p = w_.j;
      [[maybe_unused]] const int idx = i + p * m;
      P[i + p * m] = A[(k0 + i) + (size_t)(k0 + p) * n];
    }
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
      const double d = P[j + j * m];
      const bool ok = d > 0.0 && d < 1e308;
      if (!ok && tid == 0) flag_bad(status);
      const double sq = ok ? sqrt(d) : 1.0;
      const double inv = 1.0 / sq;
      for (int i = j + 1 + tid; i < m; i += kNT) P[i + j * m] *= inv;
      __syncthreads();
      if (tid == 0) P[j + j * m] = sq;
      const int w = kb - j - 1;
      for (int idx = tid; idx < w * m; idx += kNT) {
        const int i = idx % m, c = j + 1 + idx / m;
        if (i >= c) P[i + c * m] -= P[i + j * m] * P[c + j * m];
      }
      __syncthreads();
    }
    for (ColWalk w_(tid, kNT, m); w_.j < kb; w_.next()) {
      const int i = w_.i, p = w_.j;
      [[maybe_unused]] const int idx = i + p * m;
      if (i >= p) A[(k0 + i) + (size_t)(k0 + p) * n] = P[i + p * m];
    }
    // trailing update of rows/cols [k0+kb, n), lower triangle, 4x4 tiles
    const int mt = m - kb;
    const int nt = (mt + 3) / 4;
    const int ntiles = nt * (nt + 1) / 2;
    for (int t = tid; t < ntiles; t += kNT) {
      // tile (ti, tc) with ti >= tc from the linear index t
      int tc = 0, rem = t;
      while (rem >= nt - tc) { rem -= nt - tc; ++tc; }
      const int ti = tc + rem;
      double acc[4][4] = {};
      for (int p = 0; p < kb; ++p) {
        double a[4], b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = kb + ti * 4 + r;
          const int c = kb + tc * 4 + r;
          a[r] = (i < m) ? P[i + p * m] : 0.0;
          b[r] = (c < m) ? P[c + p * m] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[r][q] += a[r] * b[q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = kb + tc * 4 + q;
        if (c >= m) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = kb + ti * 4 + r;
          if (i < m && i >= c) A[(k0 + i) + (size_t)(k0 + c) * n] -= acc[r][q];
        }
      }
    }
    __syncthreads();
  }
  // mirror the Schur complement block
  const int ng = n - nI;
  for (ColWalk w_(tid, kNT, ng); w_.j < ng; w_.next()) {
    const int i = w_.i, c = w_.j;
    [[maybe_unused]] const int idx = i + c * ng;
    if (i < c) A[(nI + i) + (size_t)(nI + c) * n] = A[(nI + c) + (size_t)(nI + i) * n];
  }
}

// ---------------------------------------------------------------------------
// Constraint rows on the non-corner interface dofs of each substructure
// (C_r, n_cr x n_r): the coarse dofs of its edges, in the order of the local
// coarse dofs (after the corners).  Corner dofs are eliminated directly.
__global__ void k_build_cr(const int32_t* __restrict__ sub_inc_ptr, const int32_t* __restrict__ sub_inc,
                           const int32_t* __restrict__ inc_edge, const int32_t* __restrict__ inc_fptr,
                           const int32_t* __restrict__ inc_fpos, const int32_t* __restrict__ edge_nsc,
                           const int32_t* __restrict__ edge_ne, const int32_t* __restrict__ edge_m,
                           const int64_t* __restrict__ qoff, const double* __restrict__ Q,
                           const int32_t* __restrict__ nr, const int32_t* __restrict__ ncr,
                           const int64_t* __restrict__ croff, double* __restrict__ Cr) {
  const int s = blockIdx.x;
  const int n_r = nr[s], n_cr = ncr[s];
  double* C = Cr + croff[s];
  for (int idx = threadIdx.x; idx < n_r * n_cr; idx += kNT) C[idx] = 0.0;
  __syncthreads();
  int row = 0;
  for (int k = sub_inc_ptr[s]; k < sub_inc_ptr[s + 1]; ++k) {
    const int inc = sub_inc[k];
    const int e = inc_edge[inc];
    const int ne = edge_ne[e], m = edge_m[e], nsc = edge_nsc[e];
    const int32_t* rpos = inc_fpos + inc_fptr[inc] + nsc;
    const double* Qe = Q + qoff[e];
    for (ColWalk w_(threadIdx.x, kNT, ne); w_.j < m; w_.next()) {
      const int p = w_.i, j = w_.j;
      [[maybe_unused]] const int idx = p + j * ne;
      C[(row + j) + (size_t)rpos[p] * n_cr] = Qe[p + (size_t)j * ne];
    }
    row += m;
  }
}

// Values of the level's coarse dofs for each kernel mode of the level (the
// constants, or the rigid-body modes of elasticity; nz columns of z at stride
// zld): the next level's kernel modes (corners copy z, edge functionals apply
// their weights), nz columns of znext at stride nc.
__global__ void k_coarse_z(int nc, const int32_t* __restrict__ cd_dof, const int32_t* __restrict__ cd_col,
                           const int32_t* __restrict__ edge_ptr, const int32_t* __restrict__ edge_dof,
                           const int64_t* __restrict__ qoff, const double* __restrict__ Q,
                           const double* __restrict__ z, int nz, int zld, double* __restrict__ znext) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nc) return;
  for (int m = 0; m < nz; ++m) {
    const double* zm = z + (size_t)m * zld;
    if (cd_col[k] < 0) {
      znext[(size_t)m * nc + k] = zm[cd_dof[k]];
      continue;
    }
    const int e = cd_dof[k], j = cd_col[k];
    const int ne = edge_ptr[e + 1] - edge_ptr[e];
    const double* q = Q + qoff[e] + (size_t)j * ne;
    double acc = 0.0;
    for (int p = 0; p < ne; ++p) acc += q[p] * zm[edge_dof[edge_ptr[e] + p]];
    znext[(size_t)m * nc + k] = acc;
  }
}

// ---------------------------------------------------------------------------
// Constrained local problem on the interface of s (eqs. ML-wDi, ML-coarse):
//   min 1/2 w^T S w - g^T w  subject to  w_c = 0 (corners), C_r w_r = 0.
// With X = S_rr^{-1} C_r^T and F = C_r X:
//   T_rr = S_rr^{-1} - X F^{-1} X^T       (substructure correction operator)
//   Psi  = [[-T_rr S_rc, X F^{-1}], [I, 0]]  (energy-minimal coarse basis, C Psi = I)
//   A_c  = Psi^T S Psi                    (coarse element matrix)
__global__ void __launch_bounds__(kNT) k_constrained_factor(
    const int64_t* __restrict__ koff, const int32_t* __restrict__ loc_ptr,
    const int32_t* __restrict__ nint, const int32_t* __restrict__ nr, const int32_t* __restrict__ ncr,
    const int64_t* __restrict__ croff, const double* __restrict__ Cr, const double* __restrict__ K,
    double* __restrict__ T, const int64_t* __restrict__ toff, double* __restrict__ Psi,
    const int64_t* __restrict__ psioff, double* __restrict__ Ac, const int64_t* __restrict__ acoff,
    double* __restrict__ work, const int64_t* __restrict__ woff, int* status) {
  const int s = blockIdx.x;
  const int n = loc_ptr[s + 1] - loc_ptr[s];
  const int nI = nint[s];
  const int ng = n - nI;
  const int n_r = nr[s];
  const int n_c = ng - n_r;
  const int n_cr = ncr[s];
  const int ncs = n_c + n_cr;
  const double* S = K + koff[s] + nI + (size_t)nI * n;   // ld n, full symmetric
  const double* C = Cr + croff[s];                       // n_cr x n_r
  double* Tr = T + toff[s];                              // n_r x n_r
  double* Ps = Psi + psioff[s];                          // ng x ncs
  double* Acs = Ac + acoff[s];                           // ncs x ncs
  double* Lr = work + woff[s];                           // n_r x n_r
  double* X = Lr + (size_t)n_r * n_r;                    // n_r x n_cr
  double* F = X + (size_t)n_r * n_cr;                    // n_cr x n_cr
  double* Y = F + (size_t)n_cr * n_cr;                   // n_cr x n_r
  double* W = Y + (size_t)n_cr * n_r;                    // ng x ncs
  const int tid = threadIdx.x;

  for (ColWalk w_(tid, kNT, n_r); w_.j < n_r; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * n_r;
    Lr[idx] = S[i + (size_t)j * n];
    Tr[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  wg_potrf(Lr, n_r, n_r, status);
  wg_trsm_lower(Lr, n_r, n_r, Tr, n_r, n_r);
  wg_trsm_lower_trans(Lr, n_r, n_r, Tr, n_r, n_r);       // Tr = S_rr^{-1}
  if (n_cr > 0) {
    for (ColWalk w_(tid, kNT, n_r); w_.j < n_cr; w_.next()) {
      const int i = w_.i, j = w_.j;
      [[maybe_unused]] const int idx = i + j * n_r;
      X[idx] = C[j + (size_t)i * n_cr];
    }
    __syncthreads();
    wg_trsm_lower(Lr, n_r, n_r, X, n_r, n_cr);
    wg_trsm_lower_trans(Lr, n_r, n_r, X, n_r, n_cr);     // X = S_rr^{-1} C_r^T
    wg_gemm(false, false, n_cr, n_cr, n_r, 1.0, C, n_cr, X, n_r, 0.0, F, n_cr);
    wg_potrf(F, n_cr, n_cr, status);                    // F = Lf Lf^T
    for (ColWalk w_(tid, kNT, n_cr); w_.j < n_r; w_.next()) {
      const int i = w_.i, j = w_.j;
      [[maybe_unused]] const int idx = i + j * n_cr;
      Y[idx] = X[j + (size_t)i * n_r];
    }
    __syncthreads();
    wg_trsm_lower(F, n_cr, n_cr, Y, n_cr, n_r);         // Y = Lf^{-1} X^T
    wg_gemm(true, false, n_r, n_r, n_cr, -1.0, Y, n_cr, Y, n_cr, 1.0, Tr, n_r);   // Tr -= Y^T Y
    wg_trsm_lower_trans(F, n_cr, n_cr, Y, n_cr, n_r);   // Y = F^{-1} X^T
  }
  // Psi: rows r, corner columns = -Tr S_rc; edge columns = (F^{-1} X^T)^T
  wg_gemm(false, false, n_r, n_c, n_r, -1.0, Tr, n_r, S + (size_t)n_r * n, n, 0.0, Ps, ng);
  for (ColWalk w_(tid, kNT, n_r); w_.j < n_cr; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * n_r;
    Ps[i + (size_t)(n_c + j) * ng] = Y[j + (size_t)i * n_cr];
  }
  for (ColWalk w_(tid, kNT, n_c); w_.j < ncs; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * n_c;
    Ps[(n_r + i) + (size_t)j * ng] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  wg_gemm(false, false, ng, ncs, ng, 1.0, S, n, Ps, ng, 0.0, W, ng);            // W = S Psi
  wg_gemm(true, false, ncs, ncs, ng, 1.0, Ps, ng, W, ng, 0.0, Acs, ncs);         // A_c = Psi^T W
  // exact symmetry of A_c
  for (ColWalk w_(tid, kNT, ncs); w_.j < ncs; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * ncs;
    if (i > j) {
      const double v = 0.5 * (Acs[i + (size_t)j * ncs] + Acs[j + (size_t)i * ncs]);
      Acs[i + (size_t)j * ncs] = v;
      Acs[j + (size_t)i * ncs] = v;
    }
  }
  // exact symmetry of T_rr
  __syncthreads();
  for (ColWalk w_(tid, kNT, n_r); w_.j < n_r; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * n_r;
    if (i > j) {
      const double v = 0.5 * (Tr[i + (size_t)j * n_r] + Tr[j + (size_t)i * n_r]);
      Tr[i + (size_t)j * n_r] = v;
      Tr[j + (size_t)i * n_r] = v;
    }
  }
}

// Coarsest level (Algorithm "Multilevel BDDC", direct solve at level L):
// A_L = sum_s R_cs^T A_cs R_cs assembled in substructure order, then factored.
__device__ inline void coarsest_assemble(int nsub, int nc, const int32_t* __restrict__ cptr,
                                         const int32_t* __restrict__ cid, const double* __restrict__ Ac,
                                         const int64_t* __restrict__ acoff, double* __restrict__ AL) {
  for (int s = 0; s < nsub; ++s) {
    const int m = cptr[s + 1] - cptr[s];
    const int32_t* map = cid + cptr[s];
    const double* Ae = Ac + acoff[s];
    for (ColWalk w_(threadIdx.x, kNT, m); w_.j < m; w_.next()) {
      const int i = w_.i, j = w_.j;
      [[maybe_unused]] const int idx = i + j * m;
      AL[map[i] + (size_t)map[j] * nc] += Ae[idx];
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kNT) k_coarsest_factor(int nsub, int nc, const int32_t* __restrict__ cptr,
                                                         const int32_t* __restrict__ cid,
                                                         const double* __restrict__ Ac,
                                                         const int64_t* __restrict__ acoff,
                                                         double* __restrict__ AL, int* status) {
  for (int idx = threadIdx.x; idx < nc * nc; idx += kNT) AL[idx] = 0.0;
  __syncthreads();
  coarsest_assemble(nsub, nc, cptr, cid, Ac, acoff, AL);
  wg_potrf(AL, nc, nc, status);
}

// the same assembly into a zeroed AL, left unfactored
__global__ void __launch_bounds__(kNT) k_coarsest_assemble(int nsub, int nc, const int32_t* __restrict__ cptr,
                                                           const int32_t* __restrict__ cid,
                                                           const double* __restrict__ Ac,
                                                           const int64_t* __restrict__ acoff,
                                                           double* __restrict__ AL) {
  coarsest_assemble(nsub, nc, cptr, cid, Ac, acoff, AL);
}

// ---------------------------------------------------------------------------
// host launchers
void launch_assemble_l1(hipStream_t st, int nsub, const int64_t* koff, const int32_t* loc_ptr,
                        const int32_t* nint, const int32_t* node_el, const int32_t* sub_el_ptr,
                        const int32_t* el_gid, const int32_t* el_loc, const double* coeff,
                        const Khat16& khat, double* K, double* diagK, const int32_t* goff, int* status) {
  launch_kernel(k_assemble_l1<4, 2, Khat16>, dim3(nsub), dim3(kNT), 0, st, koff, loc_ptr, nint, node_el,
                sub_el_ptr, el_gid, el_loc, coeff, khat, K, diagK, goff, status);
}
void launch_assemble_l1_elastic(hipStream_t st, int nsub, const int64_t* koff, const int32_t* loc_ptr,
                                const int32_t* nint, const int32_t* node_el, const int32_t* sub_el_ptr,
                                const int32_t* el_gid, const int32_t* el_loc, const double* coeff,
                                const Khat64& khat, double* K, double* diagK, const int32_t* goff, int* status) {
  launch_kernel(k_assemble_l1<8, 3, Khat64>, dim3(nsub), dim3(kNT), 0, st, koff, loc_ptr, nint, node_el,
                sub_el_ptr, el_gid, el_loc, coeff, khat, K, diagK, goff, status);
}

void launch_assemble_coarse(hipStream_t st, int nsub, const int64_t* koff, const int32_t* loc_ptr,
                            const int32_t* nint, const int32_t* child_ptr, const int32_t* child_id,
                            const int32_t* child_map_off, const int32_t* child_map, const double* Ac,
                            const int64_t* acoff, const int32_t* nc_child, double* K, double* diagK,
                            const int32_t* goff) {
  launch_kernel(k_assemble_coarse, dim3(nsub), dim3(kNT), 0, st, koff, loc_ptr, nint, child_ptr,
                     child_id, child_map_off, child_map, Ac, acoff, nc_child, K, diagK, goff);
}

void launch_weights(hipStream_t st, int nflat, const int32_t* flat_iid, const int32_t* sh_ptr,
                    const int32_t* sh_flat, const double* diagK, double* delta) {
  if (nflat == 0) return;
  launch_kernel(k_weights, dim3((nflat + kNT - 1) / kNT), dim3(kNT), 0, st, nflat, flat_iid, sh_ptr,
                     sh_flat, diagK, delta);
}

void launch_partial_chol(hipStream_t st, int nsub, int nmax, const int64_t* koff, const int32_t* loc_ptr,
                         const int32_t* nint, double* K, int* status) {
  const size_t lds = sizeof(double) * (size_t)nmax * kPanel;
  launch_kernel(k_partial_chol, dim3(nsub), dim3(kNT), lds, st, koff, loc_ptr, nint, K, status);
}

size_t partial_chol_lds(int nmax) { return sizeof(double) * (size_t)nmax * kPanel; }

void launch_build_cr(hipStream_t st, int nsub, const int32_t* sub_inc_ptr, const int32_t* sub_inc,
                     const int32_t* inc_edge, const int32_t* inc_fptr, const int32_t* inc_fpos,
                     const int32_t* edge_nsc, const int32_t* edge_ne, const int32_t* edge_m,
                     const int64_t* qoff, const double* Q, const int32_t* nr, const int32_t* ncr,
                     const int64_t* croff, double* Cr) {
  launch_kernel(k_build_cr, dim3(nsub), dim3(kNT), 0, st, sub_inc_ptr, sub_inc, inc_edge, inc_fptr,
                     inc_fpos, edge_nsc, edge_ne, edge_m, qoff, Q, nr, ncr, croff, Cr);
}

void launch_coarse_z(hipStream_t st, int nc, const int32_t* cd_dof, const int32_t* cd_col,
                     const int32_t* edge_ptr, const int32_t* edge_dof, const int64_t* qoff,
                     const double* Q, const double* z, int nz, int zld, double* znext) {
  if (nc == 0) return;
  launch_kernel(k_coarse_z, dim3((nc + kNT - 1) / kNT), dim3(kNT), 0, st, nc, cd_dof, cd_col, edge_ptr, edge_dof,
                qoff, Q, z, nz, zld, znext);
}

void launch_constrained_factor(hipStream_t st, int nsub, const int64_t* koff, const int32_t* loc_ptr,
                               const int32_t* nint, const int32_t* nr, const int32_t* ncr,
                               const int64_t* croff, const double* Cr, const double* K, double* T,
                               const int64_t* toff, double* Psi, const int64_t* psioff, double* Ac,
                               const int64_t* acoff, double* work, const int64_t* woff, int* status) {
  launch_kernel(k_constrained_factor, dim3(nsub), dim3(kNT), 0, st, koff, loc_ptr, nint, nr, ncr,
                     croff, Cr, K, T, toff, Psi, psioff, Ac, acoff, work, woff, status);
}

void launch_coarsest_factor(hipStream_t st, int nsub, int nc, const int32_t* cptr, const int32_t* cid,
                            const double* Ac, const int64_t* acoff, double* AL, int* status) {
  launch_kernel(k_coarsest_factor, dim3(1), dim3(kNT), 0, st, nsub, nc, cptr, cid, Ac, acoff, AL,
                     status);
}
void launch_coarsest_assemble(hipStream_t st, int nsub, int nc, const int32_t* cptr, const int32_t* cid,
                              const double* Ac, const int64_t* acoff, double* AL) {
  BDDC_HIP(hipMemsetAsync(AL, 0, sizeof(double) * (size_t)nc * nc, st));
  launch_kernel(k_coarsest_assemble, dim3(1), dim3(kNT), 0, st, nsub, nc, cptr, cid, Ac, acoff, AL);
}

}  // namespace bddc

namespace bddc {

// Levels >= 2: explicit inverse of the interior Cholesky factor, Linv = L_II^{-1}
// (lower, n_I x n_I, ld n_I), so that the interior corrections of the apply are
// matrix-vector products.  One thread per column solves L x = e_j.
__global__ void __launch_bounds__(kNT) k_tri_inverse(const int64_t* __restrict__ koff,
                                                     const int32_t* __restrict__ loc_ptr,
                                                     const int32_t* __restrict__ nint, const double* __restrict__ K,
                                                     double* __restrict__ Linv, const int64_t* __restrict__ linvoff) {
  const int s = blockIdx.x;
  const int n = loc_ptr[s + 1] - loc_ptr[s];
  const int nI = nint[s];
  const double* L = K + koff[s];
  double* X = Linv + linvoff[s];
  for (int c = threadIdx.x; c < nI; c += kNT) {
    double* x = X + (size_t)c * nI;
    for (int i = 0; i < c; ++i) x[i] = 0.0;
    for (int i = c; i < nI; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) v -= L[i + (size_t)k * n] * x[k];
      x[i] = v / L[i + (size_t)i * n];
    }
  }
}

// The same inverse for large interiors, kTiCols columns per workgroup (grid:
// column blocks x substructures): right-looking forward substitution down the
// rows of the block, each thread holding its rows' entries of the block's
// columns in registers (row c0 + t + kNT m on thread t), the pivot row's
// finished entries handed over through LDS, the next column of L loaded while
// the current one is applied.  Every entry is formed as in k_tri_inverse:
// delta minus the products L(i,k) x(k) in increasing k (the terms above the
// column's diagonal are exact zeros), then divided by L(i,i), so the two
// kernels agree bitwise.  Interiors up to kTiRows x kNT dofs.
constexpr int kTiCols = 8;
constexpr int kTiRows = 8;

__global__ void __launch_bounds__(kNT) k_tri_inverse_cols(const int64_t* __restrict__ koff,
                                                          const int32_t* __restrict__ loc_ptr,
                                                          const int32_t* __restrict__ nint,
                                                          const double* __restrict__ K, double* __restrict__ Linv,
                                                          const int64_t* __restrict__ linvoff) {
  __shared__ double xk[2][kTiCols];
  const int s = blockIdx.y;
  const int n = loc_ptr[s + 1] - loc_ptr[s];
  const int nI = nint[s];
  const int c0 = blockIdx.x * kTiCols;
  if (c0 >= nI) return;   // (the whole workgroup)
  const int nc = min(kTiCols, nI - c0);
  const int tid = threadIdx.x;
  const double* L = K + koff[s];
  double* X = Linv + linvoff[s];
  double x[kTiRows][kTiCols];
#pragma unroll
  for (int m = 0; m < kTiRows; ++m)
#pragma unroll
    for (int j = 0; j < kTiCols; ++j) x[m][j] = (tid + kNT * m == j) ? 1.0 : 0.0;
  double lc[kTiRows], ln[kTiRows];
  auto load_col = [&](double* l, int k) {
#pragma unroll
    for (int m = 0; m < kTiRows; ++m) {
      const int i = c0 + tid + kNT * m;
      l[m] = (i > k && i < nI) ? L[i + (size_t)k * n] : 0.0;
    }
  };
  load_col(lc, c0);
  for (int k = c0; k < nI; ++k) {
    if (k + 1 < nI) load_col(ln, k + 1);
    const int r = k - c0, buf = k & 1;
    if (tid == r % kNT) {
      const double d = L[k + (size_t)k * n];
      const int mo = r / kNT;
#pragma unroll
      for (int m = 0; m < kTiRows; ++m)
        if (m == mo) {
#pragma unroll
          for (int j = 0; j < kTiCols; ++j) {
            x[m][j] = x[m][j] / d;
            xk[buf][j] = x[m][j];
          }
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kTiRows; ++m) {
      const int i = c0 + tid + kNT * m;
      if (i > k && i < nI) {
#pragma unroll
        for (int j = 0; j < kTiCols; ++j) x[m][j] -= lc[m] * xk[buf][j];
      }
    }
#pragma unroll
    for (int m = 0; m < kTiRows; ++m) lc[m] = ln[m];
  }
#pragma unroll
  for (int m = 0; m < kTiRows; ++m) {
    const int i = c0 + tid + kNT * m;
    if (i < nI)
#pragma unroll
      for (int j = 0; j < kTiCols; ++j)
        if (j < nc) X[i + (size_t)(c0 + j) * nI] = x[m][j];
  }
  for (int j = 0; j < nc; ++j)
    for (int i = tid; i < c0; i += kNT) X[i + (size_t)(c0 + j) * nI] = 0.0;
}

void launch_tri_inverse(hipStream_t st, int nsub, int nImax, const int64_t* koff, const int32_t* loc_ptr,
                        const int32_t* nint, const double* K, double* Linv, const int64_t* linvoff) {
  const char* env = getenv("BDDC_TRI_INVERSE");
  const bool cols = nImax <= kTiRows * kNT && nsub <= 65535 && !(env && std::string(env) == "rows");
  if (cols && nImax > 0)
    launch_kernel(k_tri_inverse_cols, dim3((nImax + kTiCols - 1) / kTiCols, nsub), dim3(kNT), 0, st, koff, loc_ptr,
                  nint, K, Linv, linvoff);
  else
    launch_kernel(k_tri_inverse, dim3(nsub), dim3(kNT), 0, st, koff, loc_ptr, nint, K, Linv, linvoff);
}

}  // namespace bddc

namespace bddc {

// ---------------------------------------------------------------------------
// Interior elimination with FP64 MFMA (v_mfma_f64_16x16x4f64): blocked
// right-looking Cholesky of the first nI columns of K_s.
//  * A panel of nb (<= 64) columns and all rows below its top is staged in LDS.
//  * The panel is factored in 16-column sub-panels: each thread holds one or two
//    rows of the sub-panel in registers and the sub-panel's own column entries
//    are broadcast through LDS, one step per column; the remaining panel columns
//    are then updated with MFMA from LDS.
//  * The rank-nb update of the trailing matrix runs on the matrix cores in
//    16 x 16 tiles of the lower triangle, read-modify-write in global memory;
//    operands are swapped so that 16 consecutive lanes hold 16 consecutive
//    rows of one column (coalesced).
// MFMA operand layout: lane l supplies A[l%16][l/16] and B[l/16][l%16]; register
// r of lane l holds D[l/16 + 4r][l%16].
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

constexpr int kCholNT = 512;            // threads per workgroup: 8 waves, one panel row each
constexpr int kCholRowsMax = kCholNT;   // panel rows held in registers

__global__ void __launch_bounds__(kCholNT) k_partial_chol_mfma(const int64_t* __restrict__ koff,
                                                               const int32_t* __restrict__ loc_ptr,
                                                               const int32_t* __restrict__ nint,
                                                               double* __restrict__ K, int nb, int* status) {
  extern __shared__ double P[];
  __shared__ double bc[2][16];
  constexpr int NW = kCholNT / 64;
  const int s = blockIdx.x;
  const int n = loc_ptr[s + 1] - loc_ptr[s];
  const int nI = nint[s];
  double* A = K + koff[s];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  for (int k0 = 0; k0 < nI; k0 += nb) {
    const int kb = min(nb, nI - k0);
    const int kb16 = (kb + 15) & ~15;          // panel width padded to the sub-panel width
    const int m = n - k0;                       // panel rows
    const int mp = (m + 15) & ~15;              // rows padded to the tile size
    // panel load, eight loads in flight per thread
    const int tot = mp * kb16;
    ColWalk cw(tid, kCholNT, mp);
    for (int base = tid; base < tot; base += 8 * kCholNT) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = base + u * kCholNT;
        v[u] = (idx < tot && cw.i < m && cw.j < kb) ? A[(k0 + cw.i) + (size_t)(k0 + cw.j) * n] : 0.0;
        cw.next();
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (base + u * kCholNT < tot) P[base + u * kCholNT] = v[u];
    }
    __syncthreads();
    for (int jb = 0; jb < kb; jb += 16) {
      const int w = min(16, kb - jb);
      const int ia = jb + tid;                  // sub-panel row of this thread, in registers
      double ra[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) ra[c] = ia < m ? P[ia + (jb + c) * mp] : 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if (j < w) {
          if (tid < w) bc[j & 1][tid] = ra[j];   // rows jb .. jb+w-1 are owned by threads 0 .. w-1
          __syncthreads();
          const double d = bc[j & 1][j];
          const bool ok = d > 0.0 && d < 1e308;
          if (!ok && tid == 0) flag_bad(status);
          const double sq = ok ? sqrt(d) : 1.0;
          const double inv = 1.0 / sq;
          if (ia == jb + j) ra[j] = sq;
          if (ia > jb + j && ia < m) {
            const double l = ra[j] * inv;
            ra[j] = l;
#pragma unroll
            for (int c = 0; c < 16; ++c)
              if (c > j && c < w && ia - jb >= c) ra[c] -= l * (bc[j & 1][c] * inv);
          }
        }
      }
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < w && ia < m) P[ia + (jb + c) * mp] = ra[c];
      __syncthreads();
      // remaining panel columns [jb+16, kb): P[i][c] -= sum_{p<16} P[i][jb+p] P[c][jb+p], i >= c
      const int ct0 = (jb + 16) / 16;
      const int nct = kb16 / 16 - ct0;
      const int nrt = mp / 16 - ct0;
      if (nct > 0) {
        const int ntiles = nct * nrt - nct * (nct - 1) / 2;   // row tile >= column tile
        for (int t = wave; t < ntiles; t += NW) {
          int tc = 0, rem = t;
          while (rem >= nrt - tc) { rem -= nrt - tc; ++tc; }
          const int ti = tc + rem;
          const int rrow = (ct0 + ti) * 16, rcol = (ct0 + tc) * 16;
          const int kq = lane >> 4;
          mfma_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kk = 0; kk < 16; kk += 4) {
            const double a = P[rrow + (lane & 15) + (jb + kk + kq) * mp];
            const double b = P[rcol + (lane & 15) + (jb + kk + kq) * mp];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
          }
          const int col = rcol + (lane & 15);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = rrow + (lane >> 4) + 4 * r;
            if (row < m && col < kb && row >= col) P[row + col * mp] -= acc[r];
          }
        }
      }
      __syncthreads();
    }
    for (ColWalk w_(tid, kCholNT, m); w_.j < kb; w_.next()) {
      const int i = w_.i, p = w_.j;
      [[maybe_unused]] const int idx = i + p * m;
      if (i >= p) A[(k0 + i) + (size_t)(k0 + p) * n] = P[i + p * mp];
    }
    // trailing update of rows/cols [kb, m) of the panel frame, lower tiles, two tiles per wave in flight
    const int t0 = kb;
    const int nt = (m - kb + 15) / 16;
    const int ntiles = nt * (nt + 1) / 2;
    const int kbp = (kb + 3) & ~3;
    const int kq = lane >> 4;
    for (int t = wave; t < ntiles; t += 2 * NW) {
      int ti[2], tc[2];
      bool live[2];
      double cv[2][4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int tt = t + h * NW;
        live[h] = tt < ntiles;
        int c = 0, rem = live[h] ? tt : 0;
        while (rem >= nt - c) { rem -= nt - c; ++c; }
        tc[h] = c;
        ti[h] = c + rem;
        const int row = t0 + ti[h] * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = t0 + tc[h] * 16 + kq + 4 * r;
          cv[h][r] = (live[h] && row < m && col < m && row >= col) ? A[(k0 + row) + (size_t)(k0 + col) * n] : 0.0;
        }
      }
      mfma_d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
      const int rc0 = t0 + tc[0] * 16 + (lane & 15), rr0 = t0 + ti[0] * 16 + (lane & 15);
      const int rc1 = t0 + tc[1] * 16 + (lane & 15), rr1 = t0 + ti[1] * 16 + (lane & 15);
      for (int kk = 0; kk < kbp; kk += 4) {
        const int off = (kk + kq) * mp;
        const double a0 = (rc0 < mp) ? P[rc0 + off] : 0.0;
        const double b0 = (rr0 < mp) ? P[rr0 + off] : 0.0;
        const double a1 = (rc1 < mp) ? P[rc1 + off] : 0.0;
        const double b1 = (rr1 < mp) ? P[rr1 + off] : 0.0;
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc1, 0, 0, 0);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int row = t0 + ti[h] * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = t0 + tc[h] * 16 + kq + 4 * r;
          if (live[h] && row < m && col < m && row >= col)
            A[(k0 + row) + (size_t)(k0 + col) * n] = cv[h][r] - (h == 0 ? acc0[r] : acc1[r]);
        }
      }
    }
    __syncthreads();
  }
  const int ng = n - nI;
  for (ColWalk w_(tid, kCholNT, ng); w_.j < ng; w_.next()) {
    const int i = w_.i, c = w_.j;
    [[maybe_unused]] const int idx = i + c * ng;
    if (i < c) A[(nI + i) + (size_t)(nI + c) * n] = A[(nI + c) + (size_t)(nI + i) * n];
  }
}

// panel width for substructures of at most nmax local dofs (0: not supported)
int partial_chol_mfma_nb(int nmax) {
  if (nmax > kCholRowsMax) return 0;
  const int mp = (nmax + 15) & ~15;
  int nb = (int)((160 * 1024 - 1024) / ((size_t)mp * sizeof(double)));
  nb = std::min(64, nb) & ~15;
  return nb;
}

size_t partial_chol_mfma_lds(int nmax) {
  const int mp = (nmax + 15) & ~15;
  return sizeof(double) * (size_t)mp * partial_chol_mfma_nb(nmax);
}

void launch_partial_chol_mfma(hipStream_t st, int nsub, int nmax, const int64_t* koff, const int32_t* loc_ptr,
                              const int32_t* nint, double* K, int* status) {
  const int nb = partial_chol_mfma_nb(nmax);
  launch_kernel(k_partial_chol_mfma, dim3(nsub), dim3(kCholNT), partial_chol_mfma_lds(nmax), st, koff, loc_ptr,
                nint, K, nb, status);
}

}  // namespace bddc

namespace bddc {

// ---------------------------------------------------------------------------
// LDS-resident variants of the local coarse-space factorization and of the
// interior triangular inverse: every intermediate stays in LDS, and each
// elimination step is one parallel rank-1 update between two barriers.

// In-place Gauss-Jordan inverse of an SPD matrix M (m x m, ld m) in LDS, no
// pivoting (every pivot is a Schur complement diagonal of an SPD matrix).
// tc, tr: 2m doubles of LDS scratch.
__device__ void wg_gj_inverse_spd(double* M, int m, double* tc, double* tr, int* status) {
  const int tid = threadIdx.x;
  for (int k = 0; k < m; ++k) {
    for (int i = tid; i < m; i += kNT) {
      tc[i] = M[i + (size_t)k * m];
      tr[i] = M[k + (size_t)i * m];
    }
    __syncthreads();
    const double p = tc[k];
    const bool ok = p > 0.0 && p < 1e308;
    if (!ok && tid == 0) flag_bad(status);
    const double ip = ok ? 1.0 / p : 0.0;
    for (ColWalk w_(tid, kNT, m); w_.j < m; w_.next()) {
      const int i = w_.i, j = w_.j;
      [[maybe_unused]] const int idx = i + j * m;
      double v;
      if (i == k) v = (j == k) ? ip : tr[j] * ip;
      else if (j == k) v = -tc[i] * ip;
      else v = M[idx] - tc[i] * tr[j] * ip;
      M[idx] = v;
    }
    __syncthreads();
  }
}

// The same Gauss-Jordan inverse with the matrix held in registers: thread t
// owns the entries t + u kNT (u < kGJ) of the column-major m x m matrix
// (m * m <= kGJ kNT, m <= 64).  Each step updates the owned entries from the
// pivot column and row in LDS without branches, and the owners of column / row
// k + 1 publish them into the other half of the double buffers tc, tr (halves
// of m + 64: every entry is stored, those of no use to the lane's own dump
// slot) in the same pass, so a step costs one barrier and no read-modify-write
// of LDS.  The arithmetic is that of wg_gj_inverse_spd, entry by entry
// (bitwise the same result).
constexpr int kGJ = 16;
__device__ void wg_gj_inverse_spd_regs(double* M, int m, double* tc, double* tr, int* status) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int mm = m * m;
  double v[kGJ];
  int ii[kGJ], jj[kGJ];
  ColWalk cw(tid, kNT, m);
#pragma unroll
  for (int u = 0; u < kGJ; ++u) {
    const bool in = tid + u * kNT < mm;
    v[u] = in ? M[tid + u * kNT] : 0.0;
    ii[u] = in ? cw.i : -1;
    jj[u] = in ? cw.j : -1;
    cw.next();
  }
#pragma unroll
  for (int u = 0; u < kGJ; ++u) {
    if (jj[u] == 0) tc[ii[u]] = v[u];
    if (ii[u] == 0) tr[jj[u]] = v[u];
  }
  __syncthreads();
  // (the dump slots of the two halves absorb the stores below)
  const int h = m + 64;  // half of each double buffer; entries m + lane are dump slots
  for (int k = 0; k < m; ++k) {
    const double* c = tc + (k & 1) * h;
    const double* r = tr + (k & 1) * h;
    double* cn = tc + ((k + 1) & 1) * h;
    double* rn = tr + ((k + 1) & 1) * h;
    const double p = c[k];
    const bool ok = p > 0.0 && p < 1e308;
    if (!ok && tid == 0) flag_bad(status);
    const double ip = ok ? 1.0 / p : 0.0;
    // branch-free: every case is formed and selected; entries of column /
    // row k + 1 are published, every other entry goes to the dump slot
#pragma unroll
    for (int u = 0; u < kGJ; ++u) {
      const int i = ii[u], j = jj[u];
      const double cv = c[max(i, 0)], rv = r[max(j, 0)];
      const double gen = v[u] - cv * rv * ip;
      const double rowk = rv * ip;
      const double colk = -cv * ip;
      const double x = (i == k) ? ((j == k) ? ip : rowk) : ((j == k) ? colk : gen);
      v[u] = x;
      cn[(j == k + 1 && i >= 0) ? i : m + lane] = x;
      rn[(i == k + 1) ? j : m + lane] = x;
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < kGJ; ++u)
    if (ii[u] >= 0) M[tid + u * kNT] = v[u];
  __syncthreads();
}

// the register form when the matrix fits it, else the LDS form (tc, tr: 2 (m + 64) each)
__device__ inline void wg_gj_inverse(double* M, int m, double* tc, double* tr, int* status) {
  if (m <= 64 && m * m <= kGJ * kNT) wg_gj_inverse_spd_regs(M, m, tc, tr, status);
  else wg_gj_inverse_spd(M, m, tc, tr, status);
}

// C (m x n, ldc) = alpha * op(A) op(B) + beta * C with every operand in LDS or global
__device__ inline void wg_gemm_nn(int m, int n, int k, double alpha, const double* A, int lda, const double* B, int ldb,
                                  double beta, double* C, int ldc) {
  for (ColWalk w_(threadIdx.x, kNT, m); w_.j < n; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * m;
    double acc = 0.0;
    for (int p = 0; p < k; ++p) acc += A[i + (size_t)p * lda] * B[p + (size_t)j * ldb];
    C[i + (size_t)j * ldc] = (beta == 0.0 ? 0.0 : beta * C[i + (size_t)j * ldc]) + alpha * acc;
  }
}

// LDS doubles of k_constrained_factor_lds for one substructure
__host__ __device__ inline size_t cf_lds_doubles(int ng, int n_r, int n_cr, int ncs) {
  const size_t a = (size_t)n_r * n_r + 3 * (size_t)n_r * n_cr + (size_t)n_cr * n_cr + 4 * (size_t)((n_r > n_cr ? n_r : n_cr) + 64);
  const size_t b = (size_t)ng * ncs;
  return (size_t)ng * ng + b + (a > b ? a : b);
}

// Same outputs as k_constrained_factor (T_rr, Psi, A_c), computed as
//   M = S_rr^{-1} (Gauss-Jordan), X = M C_r^T, F = C_r X, F^{-1} (Gauss-Jordan),
//   Z = X F^{-1}, T_rr = M - Z X^T (symmetrized), Psi_r = [-T_rr S_rc, Z],
//   A_c = Psi^T (S Psi) (symmetrized).
__global__ void __launch_bounds__(kNT) k_constrained_factor_lds(
    const int64_t* __restrict__ koff, const int32_t* __restrict__ loc_ptr, const int32_t* __restrict__ nint,
    const int32_t* __restrict__ nr, const int32_t* __restrict__ ncr, const int64_t* __restrict__ croff,
    const double* __restrict__ Cr, const double* __restrict__ K, double* __restrict__ T,
    const int64_t* __restrict__ toff, double* __restrict__ Psi, const int64_t* __restrict__ psioff,
    double* __restrict__ Ac, const int64_t* __restrict__ acoff, int* status) {
  extern __shared__ double sh[];
  const int s = blockIdx.x;
  const int n = loc_ptr[s + 1] - loc_ptr[s];
  const int nI = nint[s];
  const int ng = n - nI;
  const int n_r = nr[s];
  const int n_c = ng - n_r;
  const int n_cr = ncr[s];
  const int ncs = n_c + n_cr;
  const double* Sg = K + koff[s] + nI + (size_t)nI * n;  // ld n, full symmetric
  const double* C = Cr + croff[s];                       // n_cr x n_r, ld n_cr
  const int tid = threadIdx.x;
  double* S = sh;                                        // ng x ng, ld ng (staged Schur complement)
  double* Ps = S + (size_t)ng * ng;                      // ng x ncs
  double* M = Ps + (size_t)ng * ncs;                     // n_r x n_r
  double* Cl = M + (size_t)n_r * n_r;                    // n_cr x n_r
  double* X = Cl + (size_t)n_cr * n_r;                   // n_r x n_cr
  double* F = X + (size_t)n_r * n_cr;                    // n_cr x n_cr
  double* Z = F + (size_t)n_cr * n_cr;                   // n_r x n_cr
  double* tc = Z + (size_t)n_r * n_cr;
  double* tr = tc + 2 * ((n_r > n_cr ? n_r : n_cr) + 64);
  double* W = M;                                         // ng x ncs, after M .. Z are dead

  {
    // stage S and C, eight loads in flight per thread
    const int t1 = ng * ng, t2 = t1 + n_cr * n_r;
    ColWalk cw(tid, kNT, ng);
    for (int base = tid; base < t2; base += 8 * kNT) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = base + u * kNT;
        v[u] = idx < t1 ? Sg[cw.i + (size_t)cw.j * n] : (idx < t2 ? C[idx - t1] : 0.0);
        cw.next();
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = base + u * kNT;
        if (idx < t1) S[idx] = v[u];
        else if (idx < t2) Cl[idx - t1] = v[u];
      }
    }
  }
  __syncthreads();
  for (ColWalk w_(tid, kNT, n_r); w_.j < n_r; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * n_r;
    M[idx] = S[i + (size_t)j * ng];
  }
  __syncthreads();
  wg_gj_inverse(M, n_r, tc, tr, status);                 // M = S_rr^{-1}
  if (n_cr > 0) {
    for (ColWalk w_(tid, kNT, n_r); w_.j < n_cr; w_.next()) {  // X = M C^T
      const int i = w_.i, j = w_.j;
      [[maybe_unused]] const int idx = i + j * n_r;
      double acc = 0.0;
      for (int p = 0; p < n_r; ++p) acc += M[i + (size_t)p * n_r] * Cl[j + (size_t)p * n_cr];
      X[idx] = acc;
    }
    __syncthreads();
    wg_gemm_nn(n_cr, n_cr, n_r, 1.0, Cl, n_cr, X, n_r, 0.0, F, n_cr);   // F = C X
    __syncthreads();
    wg_gj_inverse_spd(F, n_cr, tc, tr, status);           // small: the LDS form
    wg_gemm_nn(n_r, n_cr, n_cr, 1.0, X, n_r, F, n_cr, 0.0, Z, n_r);     // Z = X F^{-1}
    __syncthreads();
    for (ColWalk w_(tid, kNT, n_r); w_.j < n_r; w_.next()) {   // M -= Z X^T
      const int i = w_.i, j = w_.j;
      [[maybe_unused]] const int idx = i + j * n_r;
      double acc = 0.0;
      for (int p = 0; p < n_cr; ++p) acc += Z[i + (size_t)p * n_r] * X[j + (size_t)p * n_r];
      M[idx] -= acc;
    }
    __syncthreads();
  }
  for (ColWalk w_(tid, kNT, n_r); w_.j < n_r; w_.next()) {     // exact symmetry of T_rr
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * n_r;
    if (i > j) {
      const double v = 0.5 * (M[idx] + M[j + (size_t)i * n_r]);
      M[idx] = v;
      M[j + (size_t)i * n_r] = v;
    }
  }
  __syncthreads();
  // Psi: rows r, corner columns -T_rr S_rc, edge columns Z; corner rows identity
  for (ColWalk w_(tid, kNT, n_r); w_.j < n_c; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * n_r;
    double acc = 0.0;
    for (int p = 0; p < n_r; ++p) acc += M[i + (size_t)p * n_r] * S[p + (size_t)(n_r + j) * ng];
    Ps[i + (size_t)j * ng] = -acc;
  }
  for (ColWalk w_(tid, kNT, n_r); w_.j < n_cr; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * n_r;
    Ps[i + (size_t)(n_c + j) * ng] = Z[idx];
  }
  for (ColWalk w_(tid, kNT, n_c); w_.j < ncs; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * n_c;
    Ps[(n_r + i) + (size_t)j * ng] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  double* Tr = T + toff[s];
  for (int idx = tid; idx < n_r * n_r; idx += kNT) Tr[idx] = M[idx];
  double* Pg = Psi + psioff[s];
  for (int idx = tid; idx < ng * ncs; idx += kNT) Pg[idx] = Ps[idx];
  __syncthreads();
  wg_gemm_nn(ng, ncs, ng, 1.0, S, ng, Ps, ng, 0.0, W, ng);            // W = S Psi
  __syncthreads();
  double* Acs = Ac + acoff[s];
  for (ColWalk w_(tid, kNT, ncs); w_.j < ncs; w_.next()) {     // A_c = Psi^T W, symmetrized
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * ncs;
    if (i < j) continue;
    double aij = 0.0, aji = 0.0;
    for (int p = 0; p < ng; ++p) {
      aij += Ps[p + (size_t)i * ng] * W[p + (size_t)j * ng];
      aji += Ps[p + (size_t)j * ng] * W[p + (size_t)i * ng];
    }
    const double v = (i == j) ? aij : 0.5 * (aij + aji);
    Acs[i + (size_t)j * ncs] = v;
    Acs[j + (size_t)i * ncs] = v;
  }
}

size_t constrained_factor_lds(int ng, int n_r, int n_cr, int ncs) {
  return sizeof(double) * cf_lds_doubles(ng, n_r, n_cr, ncs);
}

void launch_constrained_factor_lds(hipStream_t st, int nsub, size_t lds, const int64_t* koff, const int32_t* loc_ptr,
                                   const int32_t* nint, const int32_t* nr, const int32_t* ncr, const int64_t* croff,
                                   const double* Cr, const double* K, double* T, const int64_t* toff, double* Psi,
                                   const int64_t* psioff, double* Ac, const int64_t* acoff, int* status) {
  launch_kernel(k_constrained_factor_lds, dim3(nsub), dim3(kNT), lds, st, koff, loc_ptr, nint, nr, ncr, croff, Cr, K,
                T, toff, Psi, psioff, Ac, acoff, status);
}

// Linv = L_II^{-1} by in-place Gauss-Jordan on the lower triangle in LDS:
// step k scales row k by 1/L_kk and eliminates column k below the diagonal.
__global__ void __launch_bounds__(kNT) k_tri_inverse_lds(const int64_t* __restrict__ koff,
                                                         const int32_t* __restrict__ loc_ptr,
                                                         const int32_t* __restrict__ nint, const double* __restrict__ K,
                                                         double* __restrict__ Linv, const int64_t* __restrict__ linvoff) {
  extern __shared__ double sh[];
  const int s = blockIdx.x;
  const int n = loc_ptr[s + 1] - loc_ptr[s];
  const int m = nint[s];
  const double* L = K + koff[s];
  double* M = sh;                 // m x m, ld m (lower triangle used)
  double* rowk = M + (size_t)m * m;
  double* colk = rowk + m;
  const int tid = threadIdx.x;
  for (ColWalk w_(tid, kNT, m); w_.j < m; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * m;
    M[idx] = (i >= j) ? L[i + (size_t)j * n] : 0.0;
  }
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    const double d = 1.0 / M[k + (size_t)k * m];
    for (int c = tid; c < k; c += kNT) rowk[c] = M[k + (size_t)c * m] * d;
    for (int i = k + 1 + tid; i < m; i += kNT) colk[i] = M[i + (size_t)k * m];
    __syncthreads();
    for (int c = tid; c < k; c += kNT) M[k + (size_t)c * m] = rowk[c];
    if (tid == 0) M[k + (size_t)k * m] = d;
    const int rows = m - k - 1;
    for (ColWalk w_(tid, kNT, rows); w_.j < k + 1; w_.next()) {
      const int i = k + 1 + w_.i, c = w_.j;
      M[i + (size_t)c * m] = (c == k) ? -colk[i] * d : M[i + (size_t)c * m] - colk[i] * rowk[c];
    }
    __syncthreads();
  }
  double* X = Linv + linvoff[s];
  for (int idx = tid; idx < m * m; idx += kNT) X[idx] = M[idx];
}

size_t tri_inverse_lds(int nImax) { return sizeof(double) * ((size_t)nImax * nImax + 2 * (size_t)nImax); }

void launch_tri_inverse_lds(hipStream_t st, int nsub, int nImax, const int64_t* koff, const int32_t* loc_ptr,
                            const int32_t* nint, const double* K, double* Linv, const int64_t* linvoff) {
  launch_kernel(k_tri_inverse_lds, dim3(nsub), dim3(kNT), tri_inverse_lds(nImax), st, koff, loc_ptr, nint, K, Linv,
                linvoff);
}

}  // namespace bddc
