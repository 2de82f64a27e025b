// Adaptive setup: per-edge generalized eigenproblems (Section 3, Theorem
// "local-est"; Section 4, Theorem "adaptive"; Section 5, adaptive setup).
//
// For the adjacent pair (s, t) let F be their shared dofs: the shared corners
// (n_sc) followed by the edge dofs (n_e).  The stationary values of
//   J(w) = |(I - E) w|_S^2 / |w|_S^2     on  (I - P) W-tilde^{st}
// are computed here in a reduced but equivalent form:
//   * the jump (I-E)w vanishes off the edge, so the numerator depends only on
//     the jump j = w_s - w_t on the edge dofs:
//         N_e = D_t S_s,ee D_t + D_s S_t,ee D_s   (S_. the interface Schur
//     complements, D_. the pair weights d_s/(d_s+d_t), d the local diagonals);
//   * minimising the denominator over the non-shared dofs replaces S_s by its
//     Schur complement Shat_s onto F; with v = (shared corner values, s-edge,
//     t-edge) the denominator is v^T M v, M = P_s^T Shat_s P_s + P_t^T Shat_t P_t;
//   * if both substructures float, M has the null vector q = z|F (the
//     constant, or its coarse values at higher levels); Y = M + a q q^T with
//     any a > 0 (the role of Pi-bar in the theorem);
//   * the nonzero eigenvalues of (B^T N_e B, Y), B v = jump, are the
//     eigenvalues of G N_e with G = B Y^{-1} B^T, i.e. of H = R^T G R for
//     N_e = R R^T, and the constraint row c^s = w^T X restricted to the edge
//     is N_e j = R z for an eigenvector z of H.
// Eigenvectors with lambda > tau are selected, the constraint columns R z are
// orthonormalised by modified Gram-Schmidt, and lambda is returned in
// decreasing order.
#include <cstdlib>
#include <string>

#include "dense.hpp"
#include "kernels.hpp"

namespace bddc {

// Schur complement of the interface Schur complement S_s onto the shared
// dofs F of one (substructure, edge) incidence.  LDS holds the ng x ng matrix
// reordered as [rest | F]; eliminating `rest` leaves Shat in the trailing block.
// kGlobal: the working copy lives in a global workspace (ws + wsoff[inc])
// instead of LDS, for interfaces too large for one CU's LDS.
template <bool kGlobal>
__global__ void __launch_bounds__(kNT) k_pair_schur(
    const int32_t* __restrict__ inc_sub, const int32_t* __restrict__ inc_fptr,
    const int32_t* __restrict__ inc_fpos, const int64_t* __restrict__ koff,
    const int32_t* __restrict__ loc_ptr, const int32_t* __restrict__ nint, const double* __restrict__ K,
    const int64_t* __restrict__ inc_off, double* __restrict__ Shat, double* __restrict__ Sff, int* status,
    double* __restrict__ ws, const int64_t* __restrict__ wsoff) {
  extern __shared__ double lds_m[];
  const int inc = blockIdx.x;
  double* M;
  if constexpr (kGlobal) M = ws + wsoff[inc];
  else M = lds_m;
  const int s = inc_sub[inc];
  const int n = loc_ptr[s + 1] - loc_ptr[s];
  const int nI = nint[s];
  const int ng = n - nI;
  const double* S = K + koff[s] + nI + (size_t)nI * n;
  const int nF = inc_fptr[inc + 1] - inc_fptr[inc];
  const int32_t* fpos = inc_fpos + inc_fptr[inc];
  const int nR = ng - nF;
  int* perm = reinterpret_cast<int*>(M + (size_t)ng * ng);
  int* inF = perm + ng;
  const int tid = threadIdx.x;
  for (int a = tid; a < ng; a += kNT) inF[a] = -1;
  __syncthreads();
  for (int a = tid; a < nF; a += kNT) inF[fpos[a]] = a;
  __syncthreads();
  if (tid == 0) {
    int r = 0;
    for (int a = 0; a < ng; ++a)
      if (inF[a] < 0) perm[r++] = a;
    for (int a = 0; a < nF; ++a) perm[nR + a] = fpos[a];
  }
  __syncthreads();
  // gather, eight loads in flight per thread
  ColWalk cw(tid, kNT, ng);
  for (int base = tid; base < ng * ng; base += 8 * kNT) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * kNT;
      v[u] = idx < ng * ng ? S[perm[cw.i] + (size_t)perm[cw.j] * n] : 0.0;
      cw.next();
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (base + u * kNT < ng * ng) M[base + u * kNT] = v[u];
  }
  __syncthreads();
  double* sff = Sff + inc_off[inc];
  for (ColWalk w_(tid, kNT, nF); w_.j < nF; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * nF;
    sff[idx] = M[(nR + i) + (size_t)(nR + j) * ng];
  }
  wg_partial_potrf(M, ng, ng, nR, status);
  double* sh = Shat + inc_off[inc];
  for (ColWalk w_(tid, kNT, nF); w_.j < nF; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * nF;
    const int a = max(i, j), b = min(i, j);
    sh[idx] = M[(nR + a) + (size_t)(nR + b) * ng];
  }
}

// One edge per workgroup, everything in LDS: Y (nv x nv), X (nv x ne), R, G,
// H, V (ne x ne each), the constraint columns C (ne x ne) and small vectors.
__global__ void __launch_bounds__(kNT) k_pair_eig(
    int nedge, const int32_t* __restrict__ edge_s, const int32_t* __restrict__ edge_t,
    const int32_t* __restrict__ edge_nsc, const int32_t* __restrict__ edge_ne,
    const int32_t* __restrict__ edge_fdof, const int32_t* __restrict__ edge_fptr,
    const int32_t* __restrict__ inc_fptr, const int32_t* __restrict__ inc_fpos,
    const int32_t* __restrict__ goff, const double* __restrict__ diagK,
    const uint8_t* __restrict__ floating, const double* __restrict__ z, int nz, int zld,
    const double* __restrict__ Shat, const double* __restrict__ Sff, const int64_t* __restrict__ inc_off,
    double tau, double* __restrict__ lam_out, const int64_t* __restrict__ lamoff, double* __restrict__ Q,
    const int64_t* __restrict__ qoff, int32_t* __restrict__ nsel_out, int32_t* __restrict__ nkept_out,
    int* status) {
  extern __shared__ double lds[];
  __shared__ double red[kNT];
  const int e = blockIdx.x;
  const int s = edge_s[e], t = edge_t[e];
  const int nsc = edge_nsc[e], ne = edge_ne[e];
  const int nF = nsc + ne;
  const int nv = nsc + 2 * ne;
  const int tid = threadIdx.x;
  const int inc_s = 2 * e, inc_t = 2 * e + 1;
  const int32_t* fps = inc_fpos + inc_fptr[inc_s];
  const int32_t* fpt = inc_fpos + inc_fptr[inc_t];
  const double* Shs = Shat + inc_off[inc_s];
  const double* Sht = Shat + inc_off[inc_t];
  const double* Sfs = Sff + inc_off[inc_s];
  const double* Sft = Sff + inc_off[inc_t];

  double* Y = lds;                       // nv x nv
  double* X = Y + (size_t)nv * nv;       // nv x ne
  double* R = X + (size_t)nv * ne;       // ne x ne
  double* G = R + (size_t)ne * ne;       // ne x ne, later the constraint columns
  double* H = G + (size_t)ne * ne;       // ne x ne
  double* V = H + (size_t)ne * ne;       // ne x ne
  double* ds = V + (size_t)ne * ne;      // pair weight of s on each edge dof
  double* dt = ds + ne;                  // pair weight of t (computed directly, not as 1 - ds)
  double* cs = dt + ne;                  // rotation cosines (ne/2+1)
  double* sn = cs + (ne / 2 + 1);        // rotation sines (ne/2+1)
  double* lam = sn + (ne / 2 + 1);       // ne
  double* q = lam + ne;                  // kMaxModes x nv: the kernel modes on F in v coordinates
  int* perm = reinterpret_cast<int*>(q + (size_t)kMaxModes * nv);

  // pair weights on the edge dofs: delta_s^{st} = d_s / (d_s + d_t)
  for (int p = tid; p < ne; p += kNT) {
    const double a = diagK[goff[s] + fps[nsc + p]];
    const double b = diagK[goff[t] + fpt[nsc + p]];
    ds[p] = a / (a + b);
    dt[p] = b / (a + b);
  }
  const bool both_float = floating[s] && floating[t];
  if (both_float) {
    for (int i = tid; i < nv; i += kNT) {
      const int f = i < nsc ? i : (i < nsc + ne ? i : i - ne);
      for (int m = 0; m < nz; ++m) q[i + m * nv] = z[(size_t)m * zld + edge_fdof[edge_fptr[e] + f]];
    }
  }
  // M in the coordinates v = [shared corners | s-edge | t-edge]: s side at F
  // index i = v index i, t side at v index i (corners) or i + ne (t-edge)
  for (ColWalk w_(tid, kNT, nv); w_.j < nv; w_.next()) {
    const int vi = w_.i, vj = w_.j;
    [[maybe_unused]] const int idx = vi + vj * nv;
    double y = 0.0;
    if (vi < nF && vj < nF) y += Shs[vi + (size_t)vj * nF];
    const int ti = vi < nsc ? vi : (vi >= nsc + ne ? vi - ne : -1);
    const int tj = vj < nsc ? vj : (vj >= nsc + ne ? vj - ne : -1);
    if (ti >= 0 && tj >= 0) y += Sht[ti + (size_t)tj * nF];
    Y[idx] = y;
  }
  __syncthreads();
  if (both_float && nz == 1) {
    // Y = M + a q q^T with a = max diag(M) / |q|^2
    double nq = 0.0, amax = 0.0;
    for (int i = tid; i < nv; i += kNT) {
      nq += q[i] * q[i];
      amax = fmax(amax, Y[i + (size_t)i * nv]);
    }
    nq = wg_sum(nq, red);
    red[tid] = amax;
    __syncthreads();
    for (int w = kNT / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
      __syncthreads();
    }
    amax = red[0];
    __syncthreads();
    const double scale = amax / nq;
    for (ColWalk w_(tid, kNT, nv); w_.j < nv; w_.next()) {
      const int i = w_.i, j = w_.j;
      [[maybe_unused]] const int idx = i + j * nv;
      Y[idx] += scale * q[i] * q[j];
    }
    __syncthreads();
  } else if (both_float) {
    // several kernel modes (elasticity: the rigid-body modes common to both
    // substructures): Y = M + a sum_m q_m q_m^T over an orthonormal basis
    // (modified Gram-Schmidt) of the modes on F, a = max diag(M)
    double amax = 0.0;
    for (int i = tid; i < nv; i += kNT) amax = fmax(amax, Y[i + (size_t)i * nv]);
    red[tid] = amax;
    __syncthreads();
    for (int w = kNT / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
      __syncthreads();
    }
    amax = red[0];
    __syncthreads();
    for (int m = 0; m < nz; ++m) {
      double* qm = q + m * nv;
      for (int p = 0; p < m; ++p) {
        const double* qp = q + p * nv;
        double d = 0.0;
        for (int i = tid; i < nv; i += kNT) d += qp[i] * qm[i];
        d = wg_sum(d, red);
        for (int i = tid; i < nv; i += kNT) qm[i] -= d * qp[i];
        __syncthreads();
      }
      double nq = 0.0;
      for (int i = tid; i < nv; i += kNT) nq += qm[i] * qm[i];
      nq = wg_sum(nq, red);
      const double inv = nq > 0.0 ? 1.0 / sqrt(nq) : 0.0;
      for (int i = tid; i < nv; i += kNT) qm[i] *= inv;
      __syncthreads();
    }
    for (ColWalk w_(tid, kNT, nv); w_.j < nv; w_.next()) {
      const int i = w_.i, j = w_.j;
      [[maybe_unused]] const int idx = i + j * nv;
      double acc = 0.0;
      for (int m = 0; m < nz; ++m) acc += q[i + m * nv] * q[j + m * nv];
      Y[idx] += amax * acc;
    }
    __syncthreads();
  }
  wg_potrf(Y, nv, nv, status);
  // X = L^{-1} B^T,  B^T columns: +1 at the s-edge dof, -1 at the t-edge dof
  for (ColWalk w_(tid, kNT, nv); w_.j < ne; w_.next()) {
    const int v = w_.i, p = w_.j;
    [[maybe_unused]] const int idx = v + p * nv;
    X[idx] = (v == nsc + p) ? 1.0 : ((v == nsc + ne + p) ? -1.0 : 0.0);
  }
  __syncthreads();
  wg_trsm_lower(Y, nv, nv, X, nv, ne);
  // N_e = D_t S_s,ee D_t + D_s S_t,ee D_s  -> R (Cholesky);  G = X^T X
  for (ColWalk w_(tid, kNT, ne); w_.j < ne; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * ne;
    const double ss = Sfs[(nsc + i) + (size_t)(nsc + j) * nF];
    const double tt = Sft[(nsc + i) + (size_t)(nsc + j) * nF];
    R[idx] = dt[i] * ss * dt[j] + ds[i] * tt * ds[j];
    double g = 0.0;
    for (int v = 0; v < nv; ++v) g += X[v + (size_t)i * nv] * X[v + (size_t)j * nv];
    G[idx] = g;
  }
  __syncthreads();
  wg_potrf(R, ne, ne, status);
  for (ColWalk w_(tid, kNT, ne); w_.j < ne; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * ne;
    if (i < j) R[idx] = 0.0;
  }
  __syncthreads();
  // V = G R, then H = R^T V
  for (ColWalk w_(tid, kNT, ne); w_.j < ne; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * ne;
    double acc = 0.0;
    for (int k = j; k < ne; ++k) acc += G[i + (size_t)k * ne] * R[k + (size_t)j * ne];
    V[idx] = acc;
  }
  __syncthreads();
  for (ColWalk w_(tid, kNT, ne); w_.j < ne; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * ne;
    double acc = 0.0;
    for (int k = i; k < ne; ++k) acc += R[k + (size_t)i * ne] * V[k + (size_t)j * ne];
    H[idx] = acc;
  }
  __syncthreads();
  for (ColWalk w_(tid, kNT, ne); w_.j < ne; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * ne;
    if (i > j) {
      const double a = 0.5 * (H[idx] + H[j + (size_t)i * ne]);
      H[idx] = a;
      H[j + (size_t)i * ne] = a;
    }
    V[idx] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();

  // cyclic Jacobi with round-robin ordering of disjoint rotation pairs
  const int m = ne + (ne & 1);
  const int npair = m / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (ColWalk w_(tid, kNT, ne); w_.j < ne; w_.next()) {
      const int i = w_.i, j = w_.j;
      [[maybe_unused]] const int idx = i + j * ne;
      const double h = H[idx];
      if (i == j) dia += h * h; else off += h * h;
    }
    off = wg_sum(off, red);
    dia = wg_sum(dia, red);
    if (off <= 1e-30 * dia || ne < 2) break;
    for (int r = 0; r < m - 1; ++r) {
      for (int k = tid; k < npair; k += kNT) {
        int a = (k == 0) ? 0 : ((k - 1 + r) % (m - 1)) + 1;
        int b = ((m - 1 - k - 1 + r) % (m - 1)) + 1;
        int p = min(a, b), q2 = max(a, b);
        double c = 1.0, sv = 0.0;
        if (q2 < ne) {
          const double hpq = H[p + (size_t)q2 * ne];
          if (fabs(hpq) > 1e-300) {
            const double theta = (H[q2 + (size_t)q2 * ne] - H[p + (size_t)p * ne]) / (2.0 * hpq);
            const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            sv = tt * c;
          }
        }
        cs[k] = c;
        sn[k] = sv;
      }
      __syncthreads();
      // rows: H <- P^T H
      for (ColWalk w_(tid, kNT, npair); w_.j < ne; w_.next()) {
        const int k = w_.i, col = w_.j;
        [[maybe_unused]] const int idx = k + col * npair;
        int a = (k == 0) ? 0 : ((k - 1 + r) % (m - 1)) + 1;
        int b = ((m - 1 - k - 1 + r) % (m - 1)) + 1;
        int p = min(a, b), q2 = max(a, b);
        if (q2 >= ne) continue;
        const double c = cs[k], sv = sn[k];
        const double hp = H[p + (size_t)col * ne], hq = H[q2 + (size_t)col * ne];
        H[p + (size_t)col * ne] = c * hp - sv * hq;
        H[q2 + (size_t)col * ne] = sv * hp + c * hq;
      }
      __syncthreads();
      // columns: H <- H P, V <- V P
      for (ColWalk w_(tid, kNT, npair); w_.j < ne; w_.next()) {
        const int k = w_.i, row = w_.j;
        [[maybe_unused]] const int idx = k + row * npair;
        int a = (k == 0) ? 0 : ((k - 1 + r) % (m - 1)) + 1;
        int b = ((m - 1 - k - 1 + r) % (m - 1)) + 1;
        int p = min(a, b), q2 = max(a, b);
        if (q2 >= ne) continue;
        const double c = cs[k], sv = sn[k];
        const double hp = H[row + (size_t)p * ne], hq = H[row + (size_t)q2 * ne];
        H[row + (size_t)p * ne] = c * hp - sv * hq;
        H[row + (size_t)q2 * ne] = sv * hp + c * hq;
        const double vp = V[row + (size_t)p * ne], vq = V[row + (size_t)q2 * ne];
        V[row + (size_t)p * ne] = c * vp - sv * vq;
        V[row + (size_t)q2 * ne] = sv * vp + c * vq;
      }
      __syncthreads();
    }
  }
  // eigenvalues in decreasing order
  for (int i = tid; i < ne; i += kNT) lam[i] = H[i + (size_t)i * ne];
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < ne; ++i) perm[i] = i;
    for (int i = 1; i < ne; ++i) {
      const int key = perm[i];
      int j = i - 1;
      while (j >= 0 && lam[perm[j]] < lam[key]) { perm[j + 1] = perm[j]; --j; }
      perm[j + 1] = key;
    }
  }
  __syncthreads();
  double* lo = lam_out + lamoff[e];
  for (int i = tid; i < ne; i += kNT) lo[i] = lam[perm[i]];
  int nsel = 0;
  for (int i = 0; i < ne; ++i) nsel += (lam[perm[i]] > tau) ? 1 : 0;
  // constraint columns c_k = R z_k, k < nsel (in G), then modified Gram-Schmidt
  double* Cc = G;
  for (ColWalk w_(tid, kNT, ne); w_.j < nsel; w_.next()) {
    const int i = w_.i, k = w_.j;
    [[maybe_unused]] const int idx = i + k * ne;
    const double* zk = V + (size_t)perm[k] * ne;
    double acc = 0.0;
    for (int j = 0; j <= i; ++j) acc += R[i + (size_t)j * ne] * zk[j];
    Cc[idx] = acc;
  }
  __syncthreads();
  int kept = 0;
  double maxnorm = 0.0;
  for (int k = 0; k < nsel; ++k) {
    double* ck = Cc + (size_t)k * ne;
    for (int j = 0; j < kept; ++j) {
      const double* qj = Cc + (size_t)j * ne;
      double d = 0.0;
      for (int i = tid; i < ne; i += kNT) d += qj[i] * ck[i];
      d = wg_sum(d, red);
      for (int i = tid; i < ne; i += kNT) ck[i] -= d * qj[i];
      __syncthreads();
    }
    double nn = 0.0;
    for (int i = tid; i < ne; i += kNT) nn += ck[i] * ck[i];
    nn = sqrt(wg_sum(nn, red));
    maxnorm = fmax(maxnorm, nn);
    if (nn > 1e-10 * maxnorm && nn > 0.0) {
      double* dst = Cc + (size_t)kept * ne;
      for (int i = tid; i < ne; i += kNT) dst[i] = ck[i] / nn;
      ++kept;
    }
    __syncthreads();
  }
  double* Qe = Q + qoff[e];
  for (int idx = tid; idx < ne * nsel; idx += kNT) Qe[idx] = idx < ne * kept ? Cc[idx] : 0.0;
  if (tid == 0) {
    nsel_out[e] = nsel;
    nkept_out[e] = kept;
  }
  (void)nedge;
}

// ---------------------------------------------------------------------------
// The same eigenproblem with one wave64 per edge: every phase is spread over
// the 64 lanes and ordered by wave-level fences instead of workgroup barriers.
// The cyclic Jacobi method keeps the round-robin ordering of disjoint pairs;
// in each round a lane owns 2 x 2 blocks (row pair, column pair) of H and V
// and applies both one-sided rotations to them at once, the rotation of pair
// k being formed on the lane that owns the diagonal block (k, k).
namespace {

__device__ inline void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

__device__ inline double wv_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wv_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// lower Cholesky of the n x n matrix A (ld n) in place, one wave
__device__ void wv_potrf(double* A, int n, int* status) {
  const int lane = threadIdx.x;
  for (int j = 0; j < n; ++j) {
    const double d = A[j + j * n];
    const bool ok = d > 0.0 && d < 1e308;
    if (!ok && lane == 0) flag_bad(status);
    const double sq = ok ? sqrt(d) : 1.0;
    const double inv = 1.0 / sq;
    for (int i = j + 1 + lane; i < n; i += 64) A[i + j * n] *= inv;
    wsync();
    if (lane == 0) A[j + j * n] = sq;
    const int w = n - j - 1;
    for (ColWalk c(lane, 64, w); c.j < w; c.next())
      if (c.i >= c.j) A[(j + 1 + c.i) + (j + 1 + c.j) * n] -= A[(j + 1 + c.i) + j * n] * A[(j + 1 + c.j) + j * n];
    wsync();
  }
}

// Round-robin ordering of disjoint pairs over m (even) indices: pair k of round r.
__device__ inline void rr_pair(int k, int r, int m, int& p, int& q) {
  const int a = (k == 0) ? 0 : ((k - 1 + r) % (m - 1)) + 1;
  const int b = ((m - 1 - k - 1 + r) % (m - 1)) + 1;
  p = min(a, b);
  q = max(a, b);
}

}  // namespace

// kGlobal: the edge's working arrays live in a global workspace (ws +
// wsoff[e]) instead of LDS, for edges too long for one CU's LDS.
template <bool kGlobal>
__global__ void __launch_bounds__(64) k_pair_eig_wave(
    const int32_t* __restrict__ edge_s, const int32_t* __restrict__ edge_t,
    const int32_t* __restrict__ edge_nsc, const int32_t* __restrict__ edge_ne,
    const int32_t* __restrict__ edge_fdof, const int32_t* __restrict__ edge_fptr,
    const int32_t* __restrict__ inc_fptr, const int32_t* __restrict__ inc_fpos,
    const int32_t* __restrict__ goff, const double* __restrict__ diagK,
    const uint8_t* __restrict__ floating, const double* __restrict__ z, int nz, int zld,
    const double* __restrict__ Shat, const double* __restrict__ Sff, const int64_t* __restrict__ inc_off,
    double tau, double* __restrict__ lam_out, const int64_t* __restrict__ lamoff, double* __restrict__ Q,
    const int64_t* __restrict__ qoff, int32_t* __restrict__ nsel_out, int32_t* __restrict__ nkept_out,
    int* status, double* __restrict__ ws, const int64_t* __restrict__ wsoff) {
  extern __shared__ double lds_w[];
  const int e = blockIdx.x;
  double* lds;
  if constexpr (kGlobal) lds = ws + wsoff[e];
  else lds = lds_w;
  const int lane = threadIdx.x;
  const int s = edge_s[e], t = edge_t[e];
  const int nsc = edge_nsc[e], ne = edge_ne[e];
  const int nF = nsc + ne;
  const int nv = nsc + 2 * ne;
  const int inc_s = 2 * e, inc_t = 2 * e + 1;
  const int32_t* fps = inc_fpos + inc_fptr[inc_s];
  const int32_t* fpt = inc_fpos + inc_fptr[inc_t];
  const double* Shs = Shat + inc_off[inc_s];
  const double* Sht = Shat + inc_off[inc_t];
  const double* Sfs = Sff + inc_off[inc_s];
  const double* Sft = Sff + inc_off[inc_t];
  const int m = ne + (ne & 1);
  const int npair = m / 2;

  double* Y = lds;                        // nv x nv
  double* Xt = Y + (size_t)nv * nv;       // X^T: ne x nv (X = L^-1 B^T), entry (p, v) at p + v * ne
  double* R = Xt + (size_t)nv * ne;       // ne x ne
  double* G = R + (size_t)ne * ne;        // ne x ne, later the constraint columns
  double* H = G + (size_t)ne * ne;        // ne x ne
  double* V = H + (size_t)ne * ne;        // ne x ne
  double* ds = V + (size_t)ne * ne;       // ne
  double* dt = ds + ne;                   // ne
  double* lam = dt + ne;                  // ne
  double* q = lam + ne;                   // kMaxModes x nv
  int* perm = reinterpret_cast<int*>(q + (size_t)kMaxModes * nv);

  for (int p = lane; p < ne; p += 64) {
    const double a = diagK[goff[s] + fps[nsc + p]];
    const double b = diagK[goff[t] + fpt[nsc + p]];
    ds[p] = a / (a + b);
    dt[p] = b / (a + b);
  }
  const bool both_float = floating[s] && floating[t];
  if (both_float)
    for (int i = lane; i < nv; i += 64) {
      const int f = i < nsc ? i : (i < nsc + ne ? i : i - ne);
      for (int m = 0; m < nz; ++m) q[i + m * nv] = z[(size_t)m * zld + edge_fdof[edge_fptr[e] + f]];
    }
  for (ColWalk w_(lane, 64, nv); w_.j < nv; w_.next()) {
    const int vi = w_.i, vj = w_.j;
    double y = 0.0;
    if (vi < nF && vj < nF) y += Shs[vi + (size_t)vj * nF];
    const int ti = vi < nsc ? vi : (vi >= nsc + ne ? vi - ne : -1);
    const int tj = vj < nsc ? vj : (vj >= nsc + ne ? vj - ne : -1);
    if (ti >= 0 && tj >= 0) y += Sht[ti + (size_t)tj * nF];
    Y[vi + vj * nv] = y;
  }
  wsync();
  if (both_float && nz == 1) {
    // Y = M + a q q^T with a = max diag(M) / |q|^2
    double nq = 0.0, amax = 0.0;
    for (int i = lane; i < nv; i += 64) {
      nq += q[i] * q[i];
      amax = fmax(amax, Y[i + i * nv]);
    }
    nq = wv_sum(nq);
    amax = wv_max(amax);
    const double scale = amax / nq;
    for (ColWalk w_(lane, 64, nv); w_.j < nv; w_.next()) Y[w_.i + w_.j * nv] += scale * q[w_.i] * q[w_.j];
    wsync();
  } else if (both_float) {
    // several kernel modes: Y = M + a sum_m q_m q_m^T, q_m orthonormalised
    // (modified Gram-Schmidt), a = max diag(M)
    double amax = 0.0;
    for (int i = lane; i < nv; i += 64) amax = fmax(amax, Y[i + i * nv]);
    amax = wv_max(amax);
    for (int m = 0; m < nz; ++m) {
      double* qm = q + m * nv;
      for (int p = 0; p < m; ++p) {
        const double* qp = q + p * nv;
        double d = 0.0;
        for (int i = lane; i < nv; i += 64) d += qp[i] * qm[i];
        d = wv_sum(d);
        for (int i = lane; i < nv; i += 64) qm[i] -= d * qp[i];
        wsync();
      }
      double nq = 0.0;
      for (int i = lane; i < nv; i += 64) nq += qm[i] * qm[i];
      nq = wv_sum(nq);
      const double inv = nq > 0.0 ? 1.0 / sqrt(nq) : 0.0;
      for (int i = lane; i < nv; i += 64) qm[i] *= inv;
      wsync();
    }
    for (ColWalk w_(lane, 64, nv); w_.j < nv; w_.next()) {
      double acc = 0.0;
      for (int m = 0; m < nz; ++m) acc += q[w_.i + m * nv] * q[w_.j + m * nv];
      Y[w_.i + w_.j * nv] += amax * acc;
    }
    wsync();
  }
  wv_potrf(Y, nv, status);
  // X = L^{-1} B^T, B^T column p: +1 at the s-edge dof, -1 at the t-edge dof;
  // row by row, the lanes over the columns p
  // (each lane reads back only its own column)
  for (int v = 0; v < nv; ++v)
    for (int p = lane; p < ne; p += 64) {
      double x = (v == nsc + p) ? 1.0 : ((v == nsc + ne + p) ? -1.0 : 0.0);
      for (int k = 0; k < v; ++k) x -= Y[v + k * nv] * Xt[p + k * ne];
      Xt[p + v * ne] = x / Y[v + v * nv];
    }
  wsync();
  // N_e = D_t S_s,ee D_t + D_s S_t,ee D_s -> R;  G = X^T X
  for (ColWalk w_(lane, 64, ne); w_.j < ne; w_.next()) {
    const int i = w_.i, j = w_.j;
    const double ss = Sfs[(nsc + i) + (size_t)(nsc + j) * nF];
    const double tt = Sft[(nsc + i) + (size_t)(nsc + j) * nF];
    R[i + j * ne] = dt[i] * ss * dt[j] + ds[i] * tt * ds[j];
    double g = 0.0;
    for (int v = 0; v < nv; ++v) g += Xt[i + v * ne] * Xt[j + v * ne];
    G[i + j * ne] = g;
  }
  wsync();
  wv_potrf(R, ne, status);
  for (ColWalk w_(lane, 64, ne); w_.j < ne; w_.next())
    if (w_.i < w_.j) R[w_.i + w_.j * ne] = 0.0;
  wsync();
  // V = G R, then H = R^T V (symmetrized), V = I
  for (ColWalk w_(lane, 64, ne); w_.j < ne; w_.next()) {
    const int i = w_.i, j = w_.j;
    double acc = 0.0;
    for (int k = j; k < ne; ++k) acc += G[i + k * ne] * R[k + j * ne];
    V[i + j * ne] = acc;
  }
  wsync();
  for (ColWalk w_(lane, 64, ne); w_.j < ne; w_.next()) {
    const int i = w_.i, j = w_.j;
    double acc = 0.0;
    for (int k = i; k < ne; ++k) acc += R[k + i * ne] * V[k + j * ne];
    H[i + j * ne] = acc;
  }
  wsync();
  for (ColWalk w_(lane, 64, ne); w_.j < ne; w_.next()) {
    const int i = w_.i, j = w_.j;
    if (i > j) {
      const double a = 0.5 * (H[i + j * ne] + H[j + i * ne]);
      H[i + j * ne] = a;
      H[j + i * ne] = a;
    }
  }
  wsync();
  for (ColWalk w_(lane, 64, ne); w_.j < ne; w_.next()) V[w_.i + w_.j * ne] = (w_.i == w_.j) ? 1.0 : 0.0;
  wsync();

  // cyclic Jacobi; lane handles blocks (k, l) = (b % npair, b / npair), b = lane, lane + 64, ...
  const int nblk = npair * npair;
  for (int sweep = 0; sweep < 60 && ne >= 2; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (ColWalk w_(lane, 64, ne); w_.j < ne; w_.next()) {
      const double h = H[w_.i + w_.j * ne];
      if (w_.i == w_.j) dia += h * h; else off += h * h;
    }
    off = wv_sum(off);
    dia = wv_sum(dia);
    if (off <= 1e-30 * dia) break;
    double* cs = G;   // rotation table in the (dead) G: cos at 2k, sin at 2k + 1
    for (int r = 0; r < m - 1; ++r) {
      // the rotation of every pair from its diagonal 2 x 2 block
      for (int k = lane; k < npair; k += 64) {
        int pk, qk;
        rr_pair(k, r, m, pk, qk);
        double c = 1.0, sn = 0.0;
        if (qk < ne) {
          const double hpq = H[pk + qk * ne];
          if (fabs(hpq) > 1e-300) {
            const double theta = (H[qk + qk * ne] - H[pk + pk * ne]) / (2.0 * hpq);
            const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            sn = tt * c;
          }
        }
        cs[2 * k] = c;
        cs[2 * k + 1] = sn;
      }
      wsync();
      // every 2 x 2 block (row pair k, column pair l) of H and V: rows by
      // pair k, columns by pair l; blocks are disjoint, a lane stores only
      // what it loaded
      for (int b = lane; b < nblk; b += 64) {
        const int k = b % npair, l = b / npair;
        int pk, qk, pl, ql;
        rr_pair(k, r, m, pk, qk);
        rr_pair(l, r, m, pl, ql);
        const bool rq = qk < ne, cq = ql < ne;   // an index >= ne is the padding of odd ne
        const double ck = cs[2 * k], sk = cs[2 * k + 1], cl = cs[2 * l], sl = cs[2 * l + 1];
        const double h00 = H[pk + pl * ne];
        const double h01 = cq ? H[pk + ql * ne] : 0.0;
        const double h10 = rq ? H[qk + pl * ne] : 0.0;
        const double h11 = rq && cq ? H[qk + ql * ne] : 0.0;
        const double v00 = V[pk + pl * ne];
        const double v01 = cq ? V[pk + ql * ne] : 0.0;
        const double v10 = rq ? V[qk + pl * ne] : 0.0;
        const double v11 = rq && cq ? V[qk + ql * ne] : 0.0;
        // rows: [h0.; h1.] <- [ck h0. - sk h1.; sk h0. + ck h1.]
        const double a00 = ck * h00 - sk * h10, a01 = ck * h01 - sk * h11;
        const double a10 = sk * h00 + ck * h10, a11 = sk * h01 + ck * h11;
        // columns of H and V: [.0 .1] <- [cl .0 - sl .1, sl .0 + cl .1]
        H[pk + pl * ne] = cl * a00 - sl * a01;
        V[pk + pl * ne] = cl * v00 - sl * v01;
        if (cq) {
          H[pk + ql * ne] = sl * a00 + cl * a01;
          V[pk + ql * ne] = sl * v00 + cl * v01;
        }
        if (rq) {
          H[qk + pl * ne] = cl * a10 - sl * a11;
          V[qk + pl * ne] = cl * v10 - sl * v11;
        }
        if (rq && cq) {
          H[qk + ql * ne] = sl * a10 + cl * a11;
          V[qk + ql * ne] = sl * v10 + cl * v11;
        }
      }
      wsync();
    }
  }
  // eigenvalues in decreasing order: rank by comparison (ties by index)
  for (int i = lane; i < ne; i += 64) lam[i] = H[i + i * ne];
  wsync();
  for (int i = lane; i < ne; i += 64) {
    int rank = 0;
    for (int j = 0; j < ne; ++j) rank += (lam[j] > lam[i] || (lam[j] == lam[i] && j < i)) ? 1 : 0;
    perm[rank] = i;
  }
  wsync();
  double* lo = lam_out + lamoff[e];
  for (int i = lane; i < ne; i += 64) lo[i] = lam[perm[i]];
  int nsel = 0;
  for (int i = 0; i < ne; ++i) nsel += (lam[i] > tau) ? 1 : 0;
  // constraint columns c_k = R z_k, k < nsel (in G), then modified Gram-Schmidt
  double* Cc = G;
  for (ColWalk w_(lane, 64, ne); w_.j < nsel; w_.next()) {
    const int i = w_.i, k = w_.j;
    const double* zk = V + (size_t)perm[k] * ne;
    double acc = 0.0;
    for (int j = 0; j <= i; ++j) acc += R[i + j * ne] * zk[j];
    Cc[i + k * ne] = acc;
  }
  wsync();
  int kept = 0;
  double maxnorm = 0.0;
  for (int k = 0; k < nsel; ++k) {
    double* ck = Cc + (size_t)k * ne;
    for (int j = 0; j < kept; ++j) {
      const double* qj = Cc + (size_t)j * ne;
      double d = 0.0;
      for (int i = lane; i < ne; i += 64) d += qj[i] * ck[i];
      d = wv_sum(d);
      for (int i = lane; i < ne; i += 64) ck[i] -= d * qj[i];
      wsync();
    }
    double nn = 0.0;
    for (int i = lane; i < ne; i += 64) nn += ck[i] * ck[i];
    nn = sqrt(wv_sum(nn));
    maxnorm = fmax(maxnorm, nn);
    if (nn > 1e-10 * maxnorm && nn > 0.0) {
      double* dst = Cc + (size_t)kept * ne;
      for (int i = lane; i < ne; i += 64) dst[i] = ck[i] / nn;
      ++kept;
    }
    wsync();
  }
  double* Qe = Q + qoff[e];
  for (int idx = lane; idx < ne * nsel; idx += 64) Qe[idx] = idx < ne * kept ? Cc[idx] : 0.0;
  if (lane == 0) {
    nsel_out[e] = nsel;
    nkept_out[e] = kept;
  }
}

void launch_pair_schur(hipStream_t st, int ninc, int ngmax, const int32_t* inc_sub, const int32_t* inc_fptr,
                       const int32_t* inc_fpos, const int64_t* koff, const int32_t* loc_ptr,
                       const int32_t* nint, const double* K, const int64_t* inc_off, double* Shat,
                       double* Sff, int* status, double* ws, const int64_t* wsoff) {
  if (ninc == 0) return;
  if (ws) {
    launch_kernel(k_pair_schur<true>, dim3(ninc), dim3(kNT), 0, st, inc_sub, inc_fptr, inc_fpos, koff, loc_ptr, nint,
                  K, inc_off, Shat, Sff, status, ws, wsoff);
    return;
  }
  const size_t lds = pair_schur_lds(ngmax);
  launch_kernel(k_pair_schur<false>, dim3(ninc), dim3(kNT), lds, st, inc_sub, inc_fptr, inc_fpos, koff, loc_ptr,
                nint, K, inc_off, Shat, Sff, status, ws, wsoff);
}

size_t pair_schur_lds(int ngmax) {
  return sizeof(double) * (size_t)ngmax * ngmax + sizeof(int) * 2 * (size_t)ngmax + 64;
}

size_t pair_eig_lds(int nemax, int nvmax) {
  return sizeof(double) * ((size_t)nvmax * nvmax + (size_t)nvmax * nemax + 4 * (size_t)nemax * nemax +
                           3 * (size_t)nemax + 2 * (nemax / 2 + 1) + (size_t)kMaxModes * nvmax) +
         sizeof(int) * (nemax + 2) + 64;
}

void launch_pair_eig(hipStream_t st, int nedge, int nemax, int nvmax, const int32_t* edge_s, const int32_t* edge_t,
                     const int32_t* edge_nsc, const int32_t* edge_ne, const int32_t* edge_fdof,
                     const int32_t* edge_fptr, const int32_t* inc_fptr, const int32_t* inc_fpos,
                     const int32_t* goff, const double* diagK, const uint8_t* floating, const double* z, int nz,
                     int zld, const double* Shat, const double* Sff, const int64_t* inc_off, double tau, double* lam,
                     const int64_t* lamoff, double* Q, const int64_t* qoff, int32_t* nsel, int32_t* nkept,
                     int* status, double* ws, const int64_t* wsoff) {
  if (nedge == 0) return;
  if (ws) {
    launch_kernel(k_pair_eig_wave<true>, dim3(nedge), dim3(64), 0, st, edge_s, edge_t, edge_nsc, edge_ne, edge_fdof,
                  edge_fptr, inc_fptr, inc_fpos, goff, diagK, floating, z, nz, zld, Shat, Sff, inc_off, tau, lam, lamoff, Q,
                  qoff, nsel, nkept, status, ws, wsoff);
    return;
  }
  const char* env = getenv("BDDC_EIG_PATH");
  if (!(env && std::string(env) == "wg")) {
    launch_kernel(k_pair_eig_wave<false>, dim3(nedge), dim3(64), pair_eig_lds(nemax, nvmax), st, edge_s, edge_t,
                  edge_nsc, edge_ne, edge_fdof, edge_fptr, inc_fptr, inc_fpos, goff, diagK, floating, z, nz, zld, Shat, Sff,
                  inc_off, tau, lam, lamoff, Q, qoff, nsel, nkept, status, ws, wsoff);
    return;
  }
  launch_kernel(k_pair_eig, dim3(nedge), dim3(kNT), pair_eig_lds(nemax, nvmax), st, nedge, edge_s, edge_t,
                edge_nsc, edge_ne, edge_fdof, edge_fptr, inc_fptr, inc_fpos, goff, diagK, floating, z, nz, zld, Shat, Sff,
                inc_off, tau, lam, lamoff, Q, qoff, nsel, nkept, status);
}

}  // namespace bddc
