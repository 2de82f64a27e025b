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
// * k_pcg_*: one PCG iteration on the level-1 interface in four launches
//   (product, update/restriction, deep levels, prolongation).  Scalars
//   (alpha, beta, convergence) are recomputed by every block from the
//   per-block partial sums of the previous launch, in a fixed order, or
//   summed once by a one-block launch on large grids; results stay bitwise
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

// Substructure of workgroup b of a launch with one workgroup per
// substructure: with xcd, the workgroups of XCD k (b = k mod 8) take the
// contiguous range k q + min(k, r) + [0, q + (k < r)) of the nsub = 8 q + r
// substructures (a bijection: XCD k holds exactly that many workgroups).
__device__ inline int sub_of_block(int b, int nsub, int xcd) {
  if (!xcd) return b;
  const int q = nsub >> 3, r = nsub & 7, k = b & 7, i = b >> 3;
  return k * q + min(k, r) + i;
}

// Live columns of a blocked PCG launch: the indices of the columns not yet
// finished, in order (lc[0..nl-1]).  Snapshot form: read once by thread 0
// into LDS (for a launch that changes the flags itself).
__device__ inline int live_columns(const PcgDev& P, int* lc) {
  __shared__ int nl_s;
  if (threadIdx.x == 0) {
    int m = 0;
    for (int c = 0; c < P.nrhs; ++c)
      if (!P.sc[c].done) lc[m++] = c;
    nl_s = m;
  }
  __syncthreads();
  return nl_s;
}

// Column slots: a phase over entries a < m of every live column gives each
// column a slot of W = m rounded up to whole waves (when W <= kNT), kNT / W
// columns side by side; thread t works on entry t mod W of column
// k0 + t / W.  Entry a of a column sits on the same lane of a wave as in the
// one-column launch, so sums over a slot keep the order of wg_sum.
__device__ inline int slot_width(int m) { return ((max(m, 1) + 63) / 64) * 64; }

// wg_sum over the threads of each slot of width W (one value per thread), for
// the kNT / W slots of one pass: out[j] = sum of slot j, to every thread
__device__ inline void slot_sums(double v, int W, double* red, double* out) {
  const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  const int wpw = W >> 6;   // waves per slot
  if ((int)threadIdx.x < nw / wpw) {
    double r = 0.0;
    for (int w = threadIdx.x * wpw; w < (int)(threadIdx.x + 1) * wpw; ++w) r += red[w];
    out[threadIdx.x] = r;
  }
  __syncthreads();
}

// One block: the sum of n partials in the order of block_sum_of (bitwise the
// same value) into the scalar `which` (0 p^T S p, 1 r.r, 2 r.z of iteration
// it).  With many blocks on both sides this replaces every consuming block's
// own pass over all the partials.
// One block per column.
__global__ void __launch_bounds__(kNT) k_pcg_sum(PcgDev P, int which, int u) {
  __shared__ double red[kNT];
  const int c = blockIdx.x;
  PcgScalars* S = P.sc + c;
  if (P.sc[0].all_done || S->done) return;
  const int it = u < 0 ? 0 : P.sc[0].it_base + u;
  const double* part = which == 0 ? P.pq_part + (size_t)c * P.ld_sub
                                  : (which == 1 ? P.rr_part + (size_t)c * P.ld_sub
                                                : P.rz_part[it & 1] + (size_t)c * P.ld_blk);
  const int n = which == 2 ? P.nblk : (which == 0 ? P.npq : P.nsub1);
  // block_sum_of's additions (thread t: entries t, t + 256, ... in order, then
  // wg_sum), with up to kAll of the thread's loads issued before the first
  // addition: one memory round trip for up to kAll * 256 partials
  constexpr int kAll = 32;
  double t[kAll];
#pragma unroll
  for (int u = 0; u < kAll; ++u) {
    const int i = threadIdx.x + u * kNT;
    t[u] = i < n ? part[i] : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < kAll; ++u)
    if (threadIdx.x + u * kNT < n) acc += t[u];
  for (int i = threadIdx.x + kAll * kNT; i < n; i += kNT) acc += part[i];
  const double v = wg_sum(acc, red);
  if (threadIdx.x == 0) {
    if (which == 0) S->pqs = v;
    else if (which == 1) S->rrs = v;
    else S->rzs[it & 1] = v;
  }
}

// Tail form of the sums (finalize 2, one column): the last block of a
// producing launch to finish sums the launch's partials in the order of
// block_sum_of (bitwise the value k_pcg_sum forms) and stores the scalar, so
// the sum needs no launch of its own.  The partials are stored and read with
// agent-scope atomic accesses, which are coherent across the XCDs' L2 caches,
// so no cache maintenance is needed: a block counts itself in on an
// agent-scope counter once its partial's store has completed, and the block
// that brings the count to the grid size reads all partials, sums them and
// resets the counter for the next launch.  A launch that returns early (the
// column finished) does so in every block, and then none counts.
__device__ inline void part_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double part_load(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void tail_sum(const PcgDev& P, int which, int it, double* red) {
  __shared__ int last_s;
  __builtin_amdgcn_s_waitcnt(0);   // (the block's partial store has completed)
  __syncthreads();
  if (threadIdx.x == 0) {
    // two levels of counters (one counter per 64 bytes): block b counts in on
    // slot b mod 64; the block that completes its slot resets it and counts
    // the slot in on the top counter, so no counter sees more than 64 atomics
    unsigned* cnt = P.tail_cnt + (size_t)which * kTailStride;
    const unsigned ns = min(gridDim.x, (unsigned)kTailSlots);
    const unsigned slot = blockIdx.x % kTailSlots;
    const unsigned in_slot = (gridDim.x - slot + kTailSlots - 1) / kTailSlots;
    unsigned* sc = cnt + 16 * (1 + slot);
    int last = 0;
    if (__hip_atomic_fetch_add(sc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 == in_slot) {
      __hip_atomic_store(sc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 == ns;
    }
    last_s = last;
  }
  __syncthreads();
  if (!last_s) return;
  const double* v = which == 0 ? P.pq_part : (which == 1 ? P.rr_part : P.rz_part[it & 1]);
  const int n = which == 2 ? P.nblk : (which == 0 ? P.npq : P.nsub1);
  // the loads and additions of block_sum_of
  double acc = 0.0;
  int i = threadIdx.x;
  for (; i + 7 * kNT < n; i += 8 * kNT) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = part_load(v + i + u * kNT);
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += t[u];
  }
  for (; i < n; i += kNT) acc += part_load(v + i);
  const double sum = wg_sum(acc, red);
  if (threadIdx.x == 0) {
    PcgScalars* S = P.sc;
    if (which == 0) S->pqs = sum;
    else if (which == 1) S->rrs = sum;
    else S->rzs[it & 1] = sum;
    __hip_atomic_store(P.tail_cnt + (size_t)which * kTailStride, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Slot form of the sums (finalize 3, one column) for p^T S p and r.z.  The
// one-block sum (block_sum_of) lets thread t add the partials t, t + 256, ...
// in that order and then reduces the 256 per-thread values (wg_sum).  Here
// slot t of the producing launch is those same partials: each block counts
// itself in on its slot's counter (agent scope, about sixteen blocks per slot)
// once its partial's store has completed, and the block that completes the
// slot adds the slot's partials in that order (read with agent-scope loads)
// and stores the slot value.  Every consuming block then reduces the 256 slot
// values as wg_sum does: bitwise the one-block sum, with no launch of its own.
static_assert(kSlots == kNT, "one slot per thread of the consuming workgroup");

__device__ inline void slot_tail(const PcgDev& P, int kind, const double* part, double* slot_out, int pidx) {
  __shared__ int last_s;
  __shared__ double pv[kNT];
  __builtin_amdgcn_s_waitcnt(0);   // (the block's partial store has completed)
  __syncthreads();
  const unsigned nb = gridDim.x, slot = (unsigned)pidx % kSlots;   // (pidx: the block's partial)
  const unsigned in_slot = (nb - slot + kSlots - 1) / kSlots;
  if (threadIdx.x == 0) {
    unsigned* c = P.slot_cnt + ((size_t)kind * kSlots + slot) * 16;
    const int last = __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 == in_slot;
    if (last) __hip_atomic_store(c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last_s = last;
  }
  __syncthreads();
  if (!last_s) return;
  double acc = 0.0;   // (thread 0's)
  for (unsigned q0 = 0; q0 < in_slot; q0 += kNT) {
    const unsigned q = q0 + threadIdx.x;
    if (q < in_slot) pv[threadIdx.x] = part_load(part + slot + (size_t)q * kSlots);
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned m = min((unsigned)kNT, in_slot - q0);
      for (unsigned u = 0; u < m; ++u) acc += pv[u];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) slot_out[slot] = acc;
}

// the sum whose 256 slot values are at `slots` (every thread of the workgroup)
__device__ inline double slot_sum(const double* slots, double* red) { return wg_sum(slots[threadIdx.x], red); }
__device__ inline const double* slots_pq(const PcgDev& P) { return P.slotv; }
__device__ inline const double* slots_rz(const PcgDev& P, int it) { return P.slotv + kSlots * (1 + (it & 1)); }

__global__ void k_slot_reset(unsigned int* cnt, double* v) {
  for (int i = threadIdx.x; i < 2 * kSlots * 16; i += blockDim.x) cnt[i] = 0u;
  for (int i = threadIdx.x; i < 3 * kSlots; i += blockDim.x) v[i] = 0.0;
}

__global__ void k_tail_reset(unsigned int* cnt) {
  for (int i = threadIdx.x; i < 3 * kTailStride; i += blockDim.x) cnt[i] = 0u;
}

// the next chunk of PCG launches starts n iterations later
__global__ void k_pcg_advance(PcgScalars* sc, int n) {
  if (threadIdx.x == 0) sc[0].it_base += n;
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
// prolongation needs no pass of its own.  With several right-hand sides every
// launch loops over the columns still iterating with its operator entries
// already loaded (registers or LDS): the operators are read once per
// iteration for all columns, and each column's arithmetic is the
// single-column arithmetic.
// BF16 storage: the upper half of the IEEE binary32 pattern, rounded to
// nearest with ties to even (finite inputs only).
__device__ inline uint16_t f32_to_bf16(float x) {
  const uint32_t b = __float_as_uint(x);
  return static_cast<uint16_t>((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

template <class D, class S>
__device__ inline D widen(S v) { return static_cast<D>(v); }
template <>
__device__ inline float widen<float, uint16_t>(uint16_t v) { return bf16_to_f32(v); }
template <>
__device__ inline double widen<double, uint16_t>(uint16_t v) { return static_cast<double>(bf16_to_f32(v)); }

// Copy n values from global src (type S) to LDS dst (type D): the first kPre
// per thread are loaded into registers by fetch() (issued early, before other
// work), the rest by finish(), which also stores everything.
template <int kPre, class S = double, class D = double>
struct Prefetch {
  S v[kPre];
  const S* src;
  D* dst;
  int n;
  __device__ void fetch(const S* s, D* d, int count) {
    src = s;
    dst = d;
    n = count;
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int i = threadIdx.x + u * kNT;
      v[u] = i < n ? src[i] : S(0);
    }
  }
  __device__ void finish() {
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int i = threadIdx.x + u * kNT;
      if (i < n) dst[i] = widen<D>(v[u]);
    }
    for (int i = threadIdx.x + kPre * kNT; i < n; i += kNT) dst[i] = widen<D>(src[i]);
  }
};

// Column j of the packed lower triangle of an m x m matrix starts here.
__device__ inline int packed_col(int j, int m) { return j * m - (j * (j - 1)) / 2; }

// Entry (i, j) of a symmetric m x m matrix held as its packed lower triangle.
__device__ inline int sym_index(int i, int j, int m) {
  return i >= j ? packed_col(j, m) + (i - j) : packed_col(i, m) + (j - i);
}

// Entry (i, j) of a level-1 PCG operator: packed lower triangle, or (full)
// the whole column-major matrix, where the entries (i, j) of consecutive rows
// i are adjacent for every j
__device__ inline int op_index(int i, int j, int m, bool full) { return full ? i + j * m : sym_index(i, j, m); }

// Thread (i, c) of a row-partial product loads the entries (i, c + k nch),
// k < K, of a packed symmetric operator into registers (unconditional loads at
// clamped in-block addresses, so they issue back to back), and later forms its
// partial row sum with them.
template <int K, class T>
struct SymRowRegs {
  T v[K];
  __device__ void load(const T* A, int m, int i, int c, int nch, bool full) {
    if (m <= 0) return;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = A[op_index(i, min(c + k * nch, m - 1), m, full)];
  }
  __device__ double dot(const T* A, int m, int i, int c, int nch, const double* x, bool full) const {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = c + k * nch;
      // keeps a widening conversion here instead of right after the load
      // (which would wait for the load before the work it should overlap)
      T r = v[k];
      __asm__ volatile("" : "+v"(r));
      if (j < m) acc += static_cast<double>(r) * x[j];
    }
    // the entries past the registers in batches of 8 loads in flight
    for (int j0 = c + K * nch; j0 < m; j0 += 8 * nch) {
      T t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = A[op_index(i, min(j0 + q * nch, m - 1), m, full)];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (j0 + q * nch < m) acc += static_cast<double>(t[q]) * x[j0 + q * nch];
    }
    return acc;
  }
  // dot for nl columns of x (stride ldx) at once: each entry of the row is
  // loaded once for all of them; column k's sum is dot's, term by term
  __device__ void dot_cols(const T* A, int m, int i, int c, int nch, const double* x, int ldx, int nl, bool full,
                           double (&acc)[kMaxRhs]) const {
#pragma unroll
    for (int k = 0; k < kMaxRhs; ++k) acc[k] = 0.0;
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const int j = c + kk * nch;
      T r = v[kk];
      __asm__ volatile("" : "+v"(r));
      if (j < m) {
        const double rd = static_cast<double>(r);
#pragma unroll
        for (int k = 0; k < kMaxRhs; ++k)
          if (k < nl) acc[k] += rd * x[k * ldx + j];
      }
    }
    for (int j0 = c + K * nch; j0 < m; j0 += 8 * nch) {
      T t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = A[op_index(i, min(j0 + q * nch, m - 1), m, full)];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int j = j0 + q * nch;
        if (j < m) {
          const double a = static_cast<double>(t[q]);
#pragma unroll
          for (int k = 0; k < kMaxRhs; ++k)
            if (k < nl) acc[k] += a * x[k * ldx + j];
        }
      }
    }
  }
};

// Partial row sum over the columns c, c + nch, ... of row i of the symmetric
// m x m matrix held as its packed lower triangle A (column-major), times x.
__device__ inline double sym_row_part(const double* A, int m, int i, int c, int nch, const double* x, bool full) {
  double acc = 0.0;
  int j = c;
  if (full) {
    for (; j < m; j += nch) acc += A[i + (size_t)j * m] * x[j];
    return acc;
  }
  for (; j <= i; j += nch) acc += A[packed_col(j, m) + (i - j)] * x[j];
  const double* Ai = A + packed_col(i, m) - i;   // row i, columns j > i
  for (; j < m; j += nch) acc += Ai[j] * x[j];
  return acc;
}

// kMulti: several columns; otherwise the one column 0 (compile-time column
// offsets, uniform pointers), with the same arithmetic per column.
// The one-column instance is held to 72 registers (seven waves per SIMD, no
// spills; 84 and five waves otherwise): with one workgroup per substructure
// the launch runs in rounds of resident workgroups.
template <bool kMulti>
__global__ void __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(kMulti ? 1 : 7)))
k_pcg_matvec(LevelDev L, PcgDev P, int u) {
  extern __shared__ double sh[];
  __shared__ double red[kMaxRhs * 16];
  __shared__ double bet[kMaxRhs];
  __shared__ int lc[kMaxRhs];
  const int s = sub_of_block(blockIdx.x, L.nsub, P.xcd);
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int g0 = L.goff[s];
  const int tid = threadIdx.x;
  // thread (mi, mc) forms the partial row sums of row mi over the columns mc,
  // mc + nch, ... for every right-hand side; its entries of S_s (packed
  // symmetric) are loaded into registers before the scalars and p are
  // formed, so HBM latency overlaps that work
  const double* Sg = P.Sp + P.spoff[s];
  const int nch = max(1, kNT / max(1, ng));
  const bool narrow = ng <= kNT;
  const int mi = narrow && ng > 0 ? tid % ng : 0;
  const int mc = narrow && ng > 0 ? tid / ng : nch;
  const bool act = narrow && mc < nch;
  SymRowRegs<16, double> sv;
  if (narrow) sv.load(Sg, ng, mi, mc, nch, P.full);
  // (the flag is tested after the operator loads are issued: they are in
  // bounds either way, and the test does not delay them)
  if (P.sc[0].all_done) return;
  const int it = P.sc[0].it_base + u;
  // the live columns and their beta: every thread reads the flags and scalars
  // (uniform loads, before this launch stores anything, so they take the
  // scalar path and do not wait for the operator loads above) and writes the
  // same values to LDS, so no barrier is needed before reading them back
  // (slot sums: the one column's beta from the r.z slots of the last two
  // iterations, every thread)
  double bslot = 0.0;
  if constexpr (!kMulti) {
    if (P.fin == 3 && it >= 2 && !P.sc[0].done) {
      const double rz1 = slot_sum(slots_rz(P, it - 1), red);
      const double rz2 = slot_sum(slots_rz(P, it - 2), red);
      bslot = rz1 / rz2;
    }
  }
  int nl = 0;
  for (int c = 0; c < P.nrhs; ++c) {
    if (P.sc[c].done) continue;
    if (it >= 2 && P.fin) bet[nl] = P.fin == 3 && !kMulti ? bslot : P.sc[c].rzs[(it - 1) & 1] / P.sc[c].rzs[(it - 2) & 1];
    lc[nl++] = c;
  }
  if (nl == 0) return;
  if constexpr (!kMulti) nl = 1;   // (the one column is live here)
  auto col = [&](int k) -> int {
    if constexpr (kMulti) return lc[k];
    else return 0;
  };
  const int psz = ng + kNT;                              // part stride per column
  double* pl = sh;                                       // nl x ng
  double* part = pl + (size_t)nl * ng;                   // nl x psz
  // beta per live column from the partials (when they are not summed once)
  if (it >= 2) {
    if (!P.fin) {
      for (int k = 0; k < nl; ++k) {
        const size_t o = (size_t)col(k) * P.ld_blk;
        const double rz = block_sum_of(P.rz_part[(it - 1) & 1] + o, P.nblk, red);
        const double rz0 = block_sum_of(P.rz_part[(it - 2) & 1] + o, P.nblk, red);
        bet[k] = rz / rz0;   // every thread, the same value
      }
    }
    if (blockIdx.x == 0 && tid < nl) P.sc[col(tid)].betas[min(it - 2, kMaxHist - 1)] = bet[tid];
  }
  // p_k = z + beta p_{k-1} on the substructure's interface, every live column
  for (int t = tid; t < ng * nl; t += kNT) {
    const int k = t / ng, a = t - k * ng;
    const int f = g0 + a;
    const int gi = L.gam_iid[f];
    const bool own = P.shf4 ? P.shf4[f].x == f : L.sh_flat[L.sh_ptr[gi]] == f;
    const size_t ci = (size_t)col(k) * P.ld_if;
    const double pv = (it >= 2) ? P.z[ci + gi] + bet[k] * P.p[(it - 1) & 1][ci + gi] : P.z[ci + gi];
    pl[k * ng + a] = pv;
    if (own) P.p[it & 1][ci + gi] = pv;
  }
  __syncthreads();
  if (narrow) {
    if (act) {
      if constexpr (kMulti) {
        double acc[kMaxRhs];
        sv.dot_cols(Sg, ng, mi, mc, nch, pl, ng, nl, P.full, acc);
#pragma unroll
        for (int k = 0; k < kMaxRhs; ++k)
          if (k < nl) part[k * psz + mi + mc * ng] = acc[k];
      } else {
        part[mi + mc * ng] = sv.dot(Sg, ng, mi, mc, nch, pl, P.full);
      }
    }
  } else {
    // wide interfaces: one thread per row, every entry of S_s loaded once and
    // applied to all live columns (each column's terms in the order of
    // sym_row_part)
    for (int i = tid; i < ng; i += kNT) {
      double acc[kMulti ? kMaxRhs : 1];
#pragma unroll
      for (int k = 0; k < (kMulti ? kMaxRhs : 1); ++k) acc[k] = 0.0;
      auto term = [&](double a, int j) {
#pragma unroll
        for (int k = 0; k < (kMulti ? kMaxRhs : 1); ++k)
          if (k < nl) acc[k] += a * pl[k * ng + j];
      };
      if (P.full) {
        // eight loads in flight, then their terms in column order
        int j = 0;
        for (; j + 8 <= ng; j += 8) {
          double t[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) t[q] = Sg[i + (size_t)(j + q) * ng];
#pragma unroll
          for (int q = 0; q < 8; ++q) term(t[q], j + q);
        }
        for (; j < ng; ++j) term(Sg[i + (size_t)j * ng], j);
      } else {
        for (int j = 0; j <= i; ++j) term(Sg[packed_col(j, ng) + (i - j)], j);
        const double* Ai = Sg + packed_col(i, ng) - i;
        for (int j = i + 1; j < ng; ++j) term(Ai[j], j);
      }
#pragma unroll
      for (int k = 0; k < (kMulti ? kMaxRhs : 1); ++k)
        if (k < nl) part[k * psz + i] = acc[k];
    }
  }
  __syncthreads();
  // the local products and energies p_s^T S_s p_s, in column slots
  const int nc = narrow ? nch : 1;
  const int W = slot_width(ng);
  if (W <= kNT) {
    const int per = kNT / W;
    for (int k0 = 0; k0 < nl; k0 += per) {
      const int k = k0 + tid / W, i = tid % W;
      double e = 0.0;
      if (tid < per * W && k < nl && i < ng) {   // (threads past the last slot idle)
        double acc = 0.0;
        for (int c = 0; c < nc; ++c) acc += part[k * psz + i + c * ng];
        P.qloc[(size_t)col(k) * P.ld_flat + g0 + i] = acc;
        e = pl[k * ng + i] * acc;
      }
      slot_sums(e, W, red, bet);
      if (tid < per && k0 + tid < nl) part_store(P.pq_part + (size_t)col(k0 + tid) * P.ld_sub + s, bet[tid]);
    }
  } else {
    for (int k = 0; k < nl; ++k) {
      double* q = P.qloc + (size_t)col(k) * P.ld_flat;
      double e = 0.0;
      for (int i = tid; i < ng; i += kNT) {
        double acc = 0.0;
        for (int c = 0; c < nc; ++c) acc += part[k * psz + i + c * ng];
        q[g0 + i] = acc;
        e += pl[k * ng + i] * acc;
      }
      e = wg_sum(e, red);
      if (tid == 0) part_store(P.pq_part + (size_t)col(k) * P.ld_sub + s, e);
    }
  }
  if constexpr (!kMulti) {
    if (P.fin == 2) tail_sum(P, 0, it, red);
    if (P.fin == 3) slot_tail(P, 0, P.pq_part, P.slotv, s);
  }
}

// Storage of T_rr and Psi in the precision forms: FP64 (kPrec 0), FP32 (1),
// factored T_rr with a BF16 inverse Cholesky factor (2).  The products are
// formed in FP64 in every form: the reduced forms cut the bytes streamed per
// iteration, and FP64 arithmetic keeps the preconditioner a fixed symmetric
// operator (FP32 arithmetic measurably adds PCG iterations).
template <int kPrec> struct PrecForm;
template <> struct PrecForm<0> { using TS = double; using PS = double; };
template <> struct PrecForm<1> { using TS = float; using PS = float; };
template <> struct PrecForm<2> { using TS = uint16_t; using PS = float; };


// it >= 1: alpha, the residual update (r_k into r[it & 1]) and x update by the
// owners, the partial r.r; then the level-1 restriction of r_k (it == 0: of
// r_0 only): g = delta r_G, b = Psi^T g (ML-coarse) and da = delta T_rr g_r
// (ML-wDi, weighted for the interface average).
//   The operator's loads (packed symmetric T_rr, or the factored form's W) are
//   issued first and land in LDS while the scalars and the residual update run.
//   FP64 / FP32 forms: thread (ti, tc) forms row ti of T_rr g_r over the
//   columns tc, tc + nch, ...  Factored BF16 form: x = D^-1 g_r, v = W x,
//   v = (I - Q Q^T)^2 v, y = W^T v, T_rr g_r = D^-1 y (two passes over W).
template <int kPrec, bool kMulti>
__global__ void __launch_bounds__(kNT) k_pcg_update_restrict(LevelDev L, PcgDev P, int u, int nrmax, int ngmax,
                                                             int ncsmax) {
  using TS = typename PrecForm<kPrec>::TS;
  using PS = typename PrecForm<kPrec>::PS;
  extern __shared__ double sh[];
  __shared__ double red[kMaxRhs * 16];   // (slot sums: waves, then the per-slot results at 16)
  __shared__ double alph[kMaxRhs];
  __shared__ int lc[kMaxRhs];
  const int s = sub_of_block(blockIdx.x, L.nsub, P.xcd);
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int ng = n - L.nint[s];
  const int g0 = L.goff[s];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;   // (wave-uniform in scalar registers)
  const int n_r = L.nr[s];
  const int ncs = L.coff[s + 1] - L.coff[s];
  const int R = P.nrhs;
  const int psz = kNT + ngmax;                          // part stride per column
  double* g = sh;                                       // R x ngmax
  double* part = sh + (size_t)R * ngmax;                // R x psz
  double* dl = part + (size_t)R * psz;                  // delta on the substructure's interface (ngmax)
  double* xv = dl + ngmax;                              // factored form: x, then v (nrmax)
  float* Tl = reinterpret_cast<float*>(xv + nrmax);                       // factored form: packed W
  float* Ql = reinterpret_cast<float*>(xv + nrmax + ((size_t)nrmax * (nrmax + 1) / 2));   // Q
  float* dinv = Ql + (size_t)nrmax * ncsmax;                              // D^-1
  const int nch = max(1, kNT / max(1, n_r));
  const int ntri = n_r * (n_r + 1) / 2;
  // the operators' loads go out first and land while the scalars are formed
  constexpr int kPV = 2;
  const PS* Pg;
  if constexpr (kPrec == 0) Pg = L.Psi + L.psioff[s];
  else Pg = P.Psi32 + L.psioff[s];
  // FP64 / FP32 forms: thread (ti, tc) holds its entries of the packed
  // symmetric T_rr in registers; factored form: W staged in LDS
  const TS* Tg = nullptr;
  if constexpr (kPrec == 0) Tg = P.Tp + P.tpoff[s];
  else if constexpr (kPrec == 1) Tg = P.Tp32 + P.tpoff[s];
  const bool narrow = n_r <= kNT;
  const int ti = narrow && n_r > 0 ? tid % n_r : 0;
  const int tc = narrow && n_r > 0 ? tid / n_r : nch;
  const bool act = narrow && tc < nch;
  SymRowRegs<16, TS> tv;
  if constexpr (kPrec != 2)
    if (narrow) tv.load(Tg, n_r, ti, tc, nch, P.full);   // every thread: no divergent region to merge
  Prefetch<8, uint16_t, float> pt;
  if constexpr (kPrec == 2) pt.fetch(P.W16 + L.toff[s], reinterpret_cast<float*>(Tl), ntri);
  // (the loads are unconditional, at clamped in-block addresses, so that
  // they issue back to back; entries outside the block are never used)
  PS pv[kPV][2];
  if (ng > 0 && ncs > 0) {
#pragma unroll
    for (int m = 0; m < kPV; ++m)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = min(wave + 4 * m, ncs - 1), a = min(lane + 64 * q, ng - 1);
        pv[m][q] = Pg[a + (size_t)k * ng];
      }
  }
  // the weights of the rows' final scaling, loaded with the operators (kept
  // in LDS below, so the last phase does not wait on another load)
  const double dlv = tid < ng ? L.delta[g0 + tid] : 0.0;
  // (the flag is tested after the operator loads are issued)
  if (P.sc[0].all_done) return;
  const int it = u < 0 ? 0 : P.sc[0].it_base + u;
  if constexpr (kPrec == 2) {
    for (int a = tid; a < n_r; a += kNT) dinv[a] = P.Dinv[g0 + a];
    const int nq = n_r * P.ncr[s];
    const float* Qg = P.Q32 + P.croff[s];
    for (int a = tid; a < nq; a += kNT) Ql[a] = Qg[a];
  }
  // the live columns and their alpha (as in the product: uniform reads, the
  // same values written by every thread, no barrier)
  int nl = 0;
  for (int c = 0; c < P.nrhs; ++c) {
    if (P.sc[c].done) continue;
    if (it > 0 && P.fin && (kMulti || P.fin != 3)) alph[nl] = P.sc[c].rzs[(it - 1) & 1] / P.sc[c].pqs;
    lc[nl++] = c;
  }
  if (nl == 0) return;
  if constexpr (!kMulti) nl = 1;   // (the one column is live here)
  auto col = [&](int k) -> int {
    if constexpr (kMulti) return lc[k];
    else return 0;
  };
  // every phase below serves all live columns (column k of g / part in LDS)
  if (it == 0) {
    if constexpr (!kMulti) {
      for (int a = tid; a < ng; a += kNT) g[a] = L.delta[g0 + a] * P.r[0][L.gam_iid[g0 + a]];
    } else {
      for (int t = tid; t < ng * nl; t += kNT) {
        const int k = t / ng, a = t - k * ng;
        g[k * ngmax + a] = L.delta[g0 + a] * P.r[0][(size_t)col(k) * P.ld_if + L.gam_iid[g0 + a]];
      }
    }
  } else {
    // alpha = r.z / p^T S p per live column, from the partials when they are
    // not summed once (one column: kept in a register)
    double alpha0 = 0.0;
    if (!P.fin) {
      for (int k = 0; k < nl; ++k) {
        const double rz = block_sum_of(P.rz_part[(it - 1) & 1] + (size_t)col(k) * P.ld_blk, P.nblk, red);
        const double pq = block_sum_of(P.pq_part + (size_t)col(k) * P.ld_sub, P.npq, red);
        alph[k] = rz / pq;   // every thread, the same value
        alpha0 = rz / pq;
      }
    } else if (!kMulti) {
      if (P.fin == 3) {
        const double rz = slot_sum(slots_rz(P, it - 1), red);
        alpha0 = rz / slot_sum(slots_pq(P), red);
      } else {
        alpha0 = P.sc[0].rzs[(it - 1) & 1] / P.sc[0].pqs;
      }
    }
    const double* rold = P.r[(it - 1) & 1];
    double* rnew = P.r[it & 1];
    const double* p = P.p[it & 1];
    // r_k = r_{k-1} - alpha sum of the sharers' q; g = delta r; owners store
    // r_k and update x; partial r.r -- entry a of column k in its slot
    auto update = [&](int k, int a) {
      const int f = g0 + a;
      const int gi = L.gam_iid[f];
      const size_t ci = (size_t)col(k) * P.ld_if;
      const double* ql = P.qloc + (size_t)col(k) * P.ld_flat;
      double q = 0.0;
      bool own;
      if (P.shf4) {
        // the sharers' flat entries in one 16-byte load (-1 past the last)
        const int4 sf = P.shf4[f];
        q += ql[sf.x];
        if (sf.y >= 0) q += ql[sf.y];
        if (sf.z >= 0) q += ql[sf.z];
        if (sf.w >= 0) q += ql[sf.w];
        own = sf.x == f;
      } else {
        for (int m = L.sh_ptr[gi]; m < L.sh_ptr[gi + 1]; ++m) q += ql[L.sh_flat[m]];
        own = L.sh_flat[L.sh_ptr[gi]] == f;
      }
      const double al = kMulti ? alph[k] : alpha0;
      // the owner's x and p are loaded with r_{k-1}, before any store (the
      // compiler may not move loads across the store of r_k)
      const double ro = rold[ci + gi];
      const double xo = own ? P.x[ci + gi] : 0.0;
      const double po = own ? p[ci + gi] : 0.0;
      const double ri = ro - al * q;
      g[k * ngmax + a] = L.delta[f] * ri;
      double rr = 0.0;
      if (own) {
        rnew[ci + gi] = ri;
        P.x[ci + gi] = xo + al * po;
        rr = ri * ri;
      }
      return rr;
    };
    auto publish = [&](int k, double rr) {
      part_store(P.rr_part + (size_t)col(k) * P.ld_sub + s, rr);
      if (s == 0) {
        PcgScalars& S = P.sc[col(k)];
        S.iters = it;
        S.alphas[min(it - 1, kMaxHist - 1)] = kMulti ? alph[k] : alpha0;
      }
    };
    const int W = slot_width(ng);
    if (!kMulti) {
      // one column: entry a on thread a, as in its slot
      double rr = 0.0;
      for (int a = tid; a < ng; a += kNT) rr += update(0, a);
      rr = wg_sum(rr, red);
      if (tid == 0) publish(0, rr);
    } else if (W <= kNT) {
      const int per = kNT / W;
      double* out = red + 16;
      for (int k0 = 0; k0 < nl; k0 += per) {
        const int k = k0 + tid / W, a = tid % W;
        const double rr = (tid < per * W && k < nl && a < ng) ? update(k, a) : 0.0;   // (past the last slot: idle)
        slot_sums(rr, W, red, out);
        if (tid < per && k0 + tid < nl) publish(k0 + tid, out[tid]);
      }
    } else {
      for (int k = 0; k < nl; ++k) {
        double rr = 0.0;
        for (int a = tid; a < ng; a += kNT) rr += update(k, a);
        rr = wg_sum(rr, red);
        if (tid == 0) publish(k, rr);
      }
    }
  }
  if constexpr (kPrec == 2) pt.finish();
  if (tid < ng) dl[tid] = dlv;
  for (int a = kNT + tid; a < ng; a += kNT) dl[a] = L.delta[g0 + a];   // (wider than the workgroup)
  __syncthreads();
  // b = Psi^T g, one wave per coarse dof, every live column (several columns:
  // each entry of Psi loaded once for all of them, the same sums per column)
  if constexpr (kMulti) {
    for (int kd = wave, m = 0; kd < ncs; kd += kNT / 64, ++m) {
      double acc[kMaxRhs];
#pragma unroll
      for (int k = 0; k < kMaxRhs; ++k) acc[k] = 0.0;
      auto term = [&](double pd, int a) {
#pragma unroll
        for (int k = 0; k < kMaxRhs; ++k)
          if (k < nl) acc[k] += pd * g[k * ngmax + a];
      };
      if (m < kPV) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int a = lane + 64 * q;
          if (a < ng) term(static_cast<double>(pv[m][q]), a);
        }
        for (int a = lane + 128; a < ng; a += 64) term(static_cast<double>(Pg[a + (size_t)kd * ng]), a);
      } else {
        for (int a = lane; a < ng; a += 64) term(static_cast<double>(Pg[a + (size_t)kd * ng]), a);
      }
#pragma unroll
      for (int k = 0; k < kMaxRhs; ++k) {
        if (k >= nl) break;
        double v = acc[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (lane == 0) P.b[(size_t)col(k) * P.ld_cflat + L.coff[s] + kd] = v;
      }
    }
  } else
  for (int kd = wave, m = 0; kd < ncs; kd += kNT / 64, ++m) {
    for (int k = 0; k < nl; ++k) {
      const double* gk = g + k * ngmax;
      double acc = 0.0;
      if (m < kPV) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int a = lane + 64 * q;
          if (a < ng) acc += static_cast<double>(pv[m][q]) * gk[a];
        }
        for (int a = lane + 128; a < ng; a += 64) acc += static_cast<double>(Pg[a + (size_t)kd * ng]) * gk[a];
      } else {
        for (int a = lane; a < ng; a += 64) acc += static_cast<double>(Pg[a + (size_t)kd * ng]) * gk[a];
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
      if (lane == 0) P.b[(size_t)col(k) * P.ld_cflat + L.coff[s] + kd] = acc;
    }
  }
  if constexpr (kPrec == 2) {
    // factored form: two dependent passes over W per column
    const int n_cr = P.ncr[s];
    for (int k = 0; k < nl; ++k) {
      const double* gk = g + k * ngmax;
      double* pk = part;
      double* da = P.da + (size_t)col(k) * P.ld_flat;
      for (ColWalk w_(tid, kNT, n_r); w_.j < nch; w_.next()) {
        const int i = w_.i, c = w_.j;
        [[maybe_unused]] const int idx = i + c * n_r;
        double acc = 0.0;
        for (int j = c; j <= i; j += nch)
          acc += static_cast<double>(Tl[packed_col(j, n_r) + (i - j)]) * (gk[j] * static_cast<double>(dinv[j]));
        pk[idx] = acc;
      }
      __syncthreads();
      for (int i = tid; i < n_r; i += kNT) {
        double acc = 0.0;
        for (int c = 0; c < nch; ++c) acc += pk[i + c * n_r];
        xv[i] = acc;
      }
      __syncthreads();
      if (n_cr > 0 && wave == 0) {
        for (int rep = 0; rep < 2; ++rep)
          for (int m = 0; m < n_cr; ++m) {
            const float* q = Ql + (size_t)m * n_r;
            double d = 0.0;
            for (int a = lane; a < n_r; a += 64) d += static_cast<double>(q[a]) * xv[a];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
            for (int a = lane; a < n_r; a += 64) xv[a] -= d * static_cast<double>(q[a]);
          }
      }
      __syncthreads();
      for (ColWalk w_(tid, kNT, n_r); w_.j < nch; w_.next()) {
        const int j = w_.i, c = w_.j;
        [[maybe_unused]] const int idx = j + c * n_r;
        const int cj = packed_col(j, n_r) - j;
        double acc = 0.0;
        for (int i = j + c; i < n_r; i += nch) acc += static_cast<double>(Tl[cj + i]) * xv[i];
        pk[idx] = acc;
      }
      __syncthreads();
      for (int i = tid; i < n_r; i += kNT) {
        double acc = 0.0;
        for (int c = 0; c < nch; ++c) acc += pk[i + c * n_r];
        da[g0 + i] = dl[i] * (acc * static_cast<double>(dinv[i]));
      }
      __syncthreads();   // part and x/v are taken by the next column
    }
  } else {
    if (narrow) {
      if (act) {
        if constexpr (kMulti) {
          double acc[kMaxRhs];
          tv.dot_cols(Tg, n_r, ti, tc, nch, g, ngmax, nl, P.full, acc);
#pragma unroll
          for (int k = 0; k < kMaxRhs; ++k)
            if (k < nl) part[k * psz + ti + tc * n_r] = acc[k];
        } else {
          part[ti + tc * n_r] = tv.dot(Tg, n_r, ti, tc, nch, g, P.full);
        }
      }
    } else {
      // wide interfaces: one thread per row, each entry of T_rr loaded once
      // for all live columns (per column the order of the one-column sum)
      for (int i = tid; i < n_r; i += kNT) {
        double acc[kMulti ? kMaxRhs : 1];
#pragma unroll
        for (int k = 0; k < (kMulti ? kMaxRhs : 1); ++k) acc[k] = 0.0;
        auto term = [&](double t, int j) {
#pragma unroll
          for (int k = 0; k < (kMulti ? kMaxRhs : 1); ++k)
            if (k < nl) acc[k] += t * g[k * ngmax + j];
        };
        int j = 0;
        for (; j + 8 <= n_r; j += 8) {   // eight loads in flight, then their terms in column order
          TS t[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) t[q] = Tg[op_index(i, j + q, n_r, P.full)];
#pragma unroll
          for (int q = 0; q < 8; ++q) term(static_cast<double>(t[q]), j + q);
        }
        for (; j < n_r; ++j) term(static_cast<double>(Tg[op_index(i, j, n_r, P.full)]), j);
#pragma unroll
        for (int k = 0; k < (kMulti ? kMaxRhs : 1); ++k)
          if (k < nl) part[k * psz + i] = acc[k];
      }
    }
    __syncthreads();
    const int nc = narrow ? nch : 1;
    if constexpr (!kMulti) {
      for (int i = tid; i < n_r; i += kNT) {
        double acc = 0.0;
        for (int c = 0; c < nc; ++c) acc += part[i + c * n_r];
        P.da[g0 + i] = dl[i] * acc;
      }
    } else {
      for (int t = tid; t < n_r * nl; t += kNT) {
        const int k = t / n_r, i = t - k * n_r;
        double acc = 0.0;
        for (int c = 0; c < nc; ++c) acc += part[k * psz + i + c * n_r];
        P.da[(size_t)col(k) * P.ld_flat + g0 + i] = dl[i] * acc;
      }
    }
  }
  if constexpr (!kMulti) {
    for (int a = n_r + tid; a < ng; a += kNT) P.da[g0 + a] = 0.0;
    if (P.fin == 2 && it > 0) tail_sum(P, 1, it, red);
  } else {
    for (int t = tid; t < (ng - n_r) * nl; t += kNT) {
      const int k = t / (ng - n_r), a = n_r + t - k * (ng - n_r);
      P.da[(size_t)col(k) * P.ld_flat + g0 + a] = 0.0;
    }
  }
}

// The reduced-precision forms of the level-1 T_rr and Psi, one workgroup per
// substructure.  FP32 form: rounded copies.  Factored BF16 form: with S_rr the
// leading n_r x n_r block of S and C_r the constraint rows on the r dofs,
//   D = diag(S_rr)^(1/2),  R R^T = D^-1 S_rr D^-1 (Cholesky),  W = R^-1,
//   Q = orthonormal basis (modified Gram-Schmidt) of Y = W D^-1 C_r^T,
// so that T_rr = S_rr^-1 - S_rr^-1 C_r^T (C_r S_rr^-1 C_r^T)^-1 C_r S_rr^-1
// = D^-1 W^T (I - Q Q^T) W D^-1.  W is rounded to BF16 (packed lower
// triangle), Q and D^-1 to FP32; whatever the rounding, the applied operator
// keeps the Gram form M^T M and so stays symmetric positive semidefinite.
// LDS (doubles): A (n_r x n_r), Wm (n_r x n_r), Y (n_r x ncrmax), C (ncrmax x n_r), d (n_r).
__global__ void __launch_bounds__(kNT) k_round_factors(LevelDev L, PcgDev P, int nrmax, int ncrmax,
                                                       const double* __restrict__ Cr, int* status) {
  extern __shared__ double shf[];
  __shared__ double red[kNT];
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int n_r = L.nr[s];
  const int ncs = L.coff[s + 1] - L.coff[s];
  const int g0 = L.goff[s];
  const int tid = threadIdx.x;
  const double* Psi = L.Psi + L.psioff[s];
  float* Psi32 = const_cast<float*>(P.Psi32) + L.psioff[s];
  for (int k = tid; k < ng * ncs; k += kNT) Psi32[k] = static_cast<float>(Psi[k]);
  if (P.prec == 1) return;   // T_rr in FP32 is written by k_pack_pcg
  const int n_cr = P.ncr[s];
  double* A = shf;
  double* Wm = A + (size_t)nrmax * nrmax;
  double* Y = Wm + (size_t)nrmax * nrmax;
  double* C = Y + (size_t)nrmax * ncrmax;
  double* d = C + (size_t)ncrmax * nrmax;
  const double* Sg = L.K + L.koff[s] + nI + (size_t)nI * n;
  for (ColWalk w_(tid, kNT, n_r); w_.j < n_r; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * n_r;
    A[idx] = Sg[i + (size_t)j * n];
    Wm[idx] = (i == j) ? 1.0 : 0.0;
  }
  const double* Cg = Cr + P.croff[s];
  for (int k = tid; k < n_cr * n_r; k += kNT) C[k] = Cg[k];
  __syncthreads();
  for (int i = tid; i < n_r; i += kNT) d[i] = sqrt(A[i + (size_t)i * n_r]);
  __syncthreads();
  for (ColWalk w_(tid, kNT, n_r); w_.j < n_r; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * n_r;
    A[idx] /= d[i] * d[j];
  }
  __syncthreads();
  wg_potrf(A, n_r, n_r, status);
  wg_trsm_lower(A, n_r, n_r, Wm, n_r, n_r);          // Wm = R^-1 (lower)
  for (ColWalk w_(tid, kNT, n_r); w_.j < n_cr; w_.next()) {
    const int i = w_.i, k = w_.j;
    [[maybe_unused]] const int idx = i + k * n_r;
    double acc = 0.0;
    for (int j = 0; j <= i; ++j) acc += Wm[i + (size_t)j * n_r] * (C[k + (size_t)j * n_cr] / d[j]);
    Y[idx] = acc;
  }
  __syncthreads();
  for (int k = 0; k < n_cr; ++k) {
    double* yk = Y + (size_t)k * n_r;
    for (int m = 0; m < k; ++m) {
      const double* qm = Y + (size_t)m * n_r;
      double dot = 0.0;
      for (int i = tid; i < n_r; i += kNT) dot += qm[i] * yk[i];
      dot = wg_sum(dot, red);
      for (int i = tid; i < n_r; i += kNT) yk[i] -= dot * qm[i];
      __syncthreads();
    }
    double nn = 0.0;
    for (int i = tid; i < n_r; i += kNT) nn += yk[i] * yk[i];
    nn = sqrt(wg_sum(nn, red));
    if (!(nn > 0.0)) {
      if (tid == 0) flag_bad(status);
      nn = 1.0;
    }
    for (int i = tid; i < n_r; i += kNT) yk[i] /= nn;
    __syncthreads();
  }
  uint16_t* W16 = const_cast<uint16_t*>(P.W16) + L.toff[s];
  for (ColWalk w_(tid, kNT, n_r); w_.j < n_r; w_.next()) {
    const int i = w_.i, j = w_.j;
    if (i >= j) W16[packed_col(j, n_r) + (i - j)] = f32_to_bf16(static_cast<float>(Wm[i + (size_t)j * n_r]));
  }
  float* Q32 = const_cast<float*>(P.Q32) + P.croff[s];
  for (int k = tid; k < n_cr * n_r; k += kNT) Q32[k] = static_cast<float>(Y[k]);
  float* Dv = const_cast<float*>(P.Dinv) + g0;
  for (int i = tid; i < n_r; i += kNT) Dv[i] = static_cast<float>(1.0 / d[i]);
}

// The level-1 operators of the PCG iteration as packed lower triangles,
// one workgroup per substructure: S_s always, T_rr in FP64 or FP32 by form.
__global__ void __launch_bounds__(kNT) k_pack_pcg(LevelDev L, PcgDev P) {
  const int s = blockIdx.x;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int n_r = L.nr[s];
  const double* S = L.K + L.koff[s] + nI + (size_t)nI * n;
  double* Sp = const_cast<double*>(P.Sp) + P.spoff[s];
  const int lds_ = P.fullpad ? pad_ld(ng, 8) : ng;
  for (ColWalk w_(threadIdx.x, kNT, ng); w_.j < ng; w_.next())
    if (P.full || w_.i >= w_.j) Sp[op_index(w_.i, w_.j, lds_, P.full)] = S[w_.i + (size_t)w_.j * n];
  if (P.prec == 2) return;
  const double* T = L.T + L.toff[s];
  const int ldt = P.fullpad ? pad_ld(n_r, P.prec == 0 ? 8 : 4) : n_r;
  for (ColWalk w_(threadIdx.x, kNT, n_r); w_.j < n_r; w_.next()) {
    if (!P.full && w_.i < w_.j) continue;
    const int k = P.full ? op_index(w_.i, w_.j, ldt, true) : op_index(w_.i, w_.j, n_r, false);
    const double v = T[w_.i + (size_t)w_.j * n_r];
    if (P.prec == 0) const_cast<double*>(P.Tp)[P.tpoff[s] + k] = v;
    else const_cast<float*>(P.Tp32)[P.tpoff[s] + k] = static_cast<float>(v);
  }
}

// Convergence test on r.r (every block takes the same decision; block 0
// records it), then per interface dof z = sum over sharers of delta T_rr g plus
// the dof's row of the delta-weighted coarse basis times u_c  (ML-uBi-1), and
// the per-block partial of r_k . z.
template <bool kMulti>
__global__ void __launch_bounds__(kNT) k_pcg_prolong_post(LevelDev L, PcgDev P, int u) {
  __shared__ double red[kMaxRhs * 16];
  __shared__ int lc[kMaxRhs];
  __shared__ int gc[kMaxRhs];
  __shared__ int ngo_s;
  if (P.sc[0].all_done) return;
  const int it = u < 0 ? 0 : P.sc[0].it_base + u;
  const bool check = it > 0;
  const int parity = it & 1;
  int ngo;
  if constexpr (kMulti) {
    // the columns' states on entry (block 0 updates them below)
    const int nl = live_columns(P, lc);
    // convergence test on r.r per live column; gc = the columns still going
    __shared__ double rrv[kMaxRhs];
    if (check) {
      if (P.fin) {
        if (threadIdx.x < nl) rrv[threadIdx.x] = P.sc[lc[threadIdx.x]].rrs;
      } else {
        for (int k = 0; k < nl; ++k) {
          const double rr = block_sum_of(P.rr_part + (size_t)lc[k] * P.ld_sub, P.nsub1, red);
          if (threadIdx.x == 0) rrv[k] = rr;
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int m = 0;
        for (int k = 0; k < nl; ++k) {
          PcgScalars* S = P.sc + lc[k];
          const bool conv = rrv[k] <= S->thr2;
          const bool maxed = S->iters >= S->maxit;
          if (blockIdx.x == 0) {
            S->rr = rrv[k];
            if (conv || maxed) S->done = conv ? 1 : 2;
          }
          if (!(conv || maxed)) gc[m++] = lc[k];
        }
        ngo_s = m;
      }
    } else if (threadIdx.x == 0) {
      for (int k = 0; k < nl; ++k) gc[k] = lc[k];
      ngo_s = nl;
    }
    __syncthreads();
    ngo = ngo_s;
    if (ngo == 0) {
      if (blockIdx.x == 0 && threadIdx.x == 0) P.sc[0].all_done = 1;
      return;
    }
  } else {
    // one column: every thread takes the same decision from the same values
    // (a wave that sees the flag raised by block 0 in this launch returns, as
    // block 0 itself does)
    PcgScalars* S = P.sc;
    if (S->done) return;
    if (check) {
      const double rr = P.fin ? S->rrs : block_sum_of(P.rr_part, P.nsub1, red);
      const bool conv = rr <= S->thr2;
      const bool maxed = S->iters >= S->maxit;
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        S->rr = rr;
        if (conv || maxed) {
          S->done = conv ? 1 : 2;
          S->all_done = 1;
        }
      }
      if (conv || maxed) return;
    }
    ngo = 1;
  }
  auto gcol = [&](int k) -> int {
    if constexpr (kMulti) return gc[k];
    else return 0;
  };
  // z = sum over the sharers of delta T_rr g plus the averaged coarse basis
  // row times u_c: eight lanes per interface dof, fixed-order reduction over
  // the eight; the partial r.z of each going column is reduced as wg_sum does
  // (per wave here, over the waves below)
  const int gi = (blockIdx.x * kNT + threadIdx.x) >> 3;
  const int sub = threadIdx.x & 7;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = kNT / 64;
  // (several columns: the sharer and coarse-row entries are loaded once for
  // all of them, each column's terms in the same order)
  double accs[kMulti ? kMaxRhs : 1];
  if constexpr (kMulti) {
#pragma unroll
    for (int k = 0; k < kMaxRhs; ++k) accs[k] = 0.0;
    if (gi < P.nif) {
      const int k0 = L.sh_ptr[gi], k1 = L.sh_ptr[gi + 1];
      for (int m = k0 + sub; m < k1; m += 8) {
        const int fl = L.sh_flat[m];
#pragma unroll
        for (int k = 0; k < kMaxRhs; ++k)
          if (k < ngo) accs[k] += P.da[(size_t)gcol(k) * P.ld_flat + fl];
      }
      for (int j = P.phi_ptr[gi] + sub; j < P.phi_ptr[gi + 1]; j += 8) {
        const double w = P.phi_w[j];
        const int id = P.phi_ids[j];
#pragma unroll
        for (int k = 0; k < kMaxRhs; ++k)
          if (k < ngo) accs[k] += w * P.uc[(size_t)gcol(k) * P.ld_coarse + id];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < (kMulti ? kMaxRhs : 1); ++k) {
    if (k >= ngo) break;
    const size_t ci = (size_t)gcol(k) * P.ld_if;
    double acc = 0.0;
    if constexpr (kMulti) {
      acc = accs[k];
    } else if (gi < P.nif) {
      const double* da = P.da + (size_t)gcol(k) * P.ld_flat;
      const double* uc = P.uc + (size_t)gcol(k) * P.ld_coarse;
      const int k0 = L.sh_ptr[gi], k1 = L.sh_ptr[gi + 1];
      for (int m = k0 + sub; m < k1; m += 8) acc += da[L.sh_flat[m]];
      for (int j = P.phi_ptr[gi] + sub; j < P.phi_ptr[gi + 1]; j += 8) acc += P.phi_w[j] * uc[P.phi_ids[j]];
    }
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 4);
    double rz = 0.0;
    if (gi < P.nif && sub == 0) {
      P.z[ci + gi] = acc;
      rz = acc * P.r[parity][ci + gi];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) rz += __shfl_xor(rz, o, 64);
    if (lane == 0) red[k * 16 + wave] = rz;
  }
  __syncthreads();
  if ((int)threadIdx.x < ngo) {
    double r = 0.0;
    for (int w = 0; w < nw; ++w) r += red[threadIdx.x * 16 + w];
    part_store(P.rz_part[parity] + (size_t)gcol(threadIdx.x) * P.ld_blk + blockIdx.x, r);
  }
  if constexpr (!kMulti) {
    if (P.fin == 2) tail_sum(P, 2, it, red);
    if (P.fin == 3) slot_tail(P, 1, P.rz_part[parity], P.slotv + kSlots * (1 + parity), blockIdx.x);
  }
}

// Rows of the averaged coarse basis: for interface dof gi, in sharer order,
// the coarse ids and delta_s(gi) Psi_s(row of gi, :) of every sharer s; with
// psi32, Psi is taken as its FP32 copy so that prolongation and restriction
// use the same basis.
__global__ void __launch_bounds__(kNT) k_build_phi(LevelDev L, int nif, const int32_t* __restrict__ sub_of_flat,
                                                   const int32_t* __restrict__ phi_ptr, int32_t* __restrict__ phi_ids,
                                                   double* __restrict__ phi_w, const float* __restrict__ psi32) {
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
    const float* Pf = psi32 ? psi32 + L.psioff[t] : nullptr;
    for (int k = 0; k < ncst; ++k) {
      phi_ids[j] = L.cid[L.coff[t] + k];
      const double w = Pf ? static_cast<double>(Pf[at + (size_t)k * ngt]) : Pt[at + (size_t)k * ngt];
      phi_w[j++] = L.delta[f] * w;
    }
  }
}

void launch_pcg_matvec(hipStream_t st, const LevelDev& L, int ngmax, const PcgDev& P, int u) {
  const size_t lds = sizeof(double) * (size_t)P.nrhs * ((size_t)ngmax + kNT + ngmax);
  if (P.nrhs > 1)
    launch_kernel(k_pcg_matvec<true>, dim3(L.nsub), dim3(kNT), lds, st, L, P, u);
  else
    launch_kernel(k_pcg_matvec<false>, dim3(L.nsub), dim3(kNT), lds, st, L, P, u);
}
void launch_pcg_sum(hipStream_t st, const PcgDev& P, int which, int u) {
  launch_kernel(k_pcg_sum, dim3(P.nrhs), dim3(kNT), 0, st, P, which, u);
}
void launch_slot_reset(hipStream_t st, const PcgDev& P) {
  launch_kernel(k_slot_reset, dim3(1), dim3(256), 0, st, P.slot_cnt, P.slotv);
}
void launch_tail_reset(hipStream_t st, const PcgDev& P) {
  launch_kernel(k_tail_reset, dim3(1), dim3(256), 0, st, P.tail_cnt);
}
void launch_pcg_advance(hipStream_t st, const PcgDev& P, int n) {
  launch_kernel(k_pcg_advance, dim3(1), dim3(64), 0, st, P.sc, n);
}
void launch_pcg_update_restrict(hipStream_t st, const LevelDev& L, int ngmax, int nrmax, int ncsmax, const PcgDev& P,
                                int u) {
  // doubles: g | part per column | delta; factored form also: x/v (doubles) | W | Q | D^-1 (floats)
  size_t lds = sizeof(double) * ((size_t)P.nrhs * ((size_t)ngmax + kNT + ngmax) + ngmax);
  if (P.prec == 2)
    lds += sizeof(double) * (nrmax + (size_t)nrmax * (nrmax + 1) / 2) +
           sizeof(float) * ((size_t)nrmax * ncsmax + nrmax);
  auto go = [&](auto kern) { launch_kernel(kern, dim3(L.nsub), dim3(kNT), lds, st, L, P, u, nrmax, ngmax, ncsmax); };
  const bool multi = P.nrhs > 1;
  if (P.prec == 0)
    multi ? go(k_pcg_update_restrict<0, true>) : go(k_pcg_update_restrict<0, false>);
  else if (P.prec == 1)
    multi ? go(k_pcg_update_restrict<1, true>) : go(k_pcg_update_restrict<1, false>);
  else
    multi ? go(k_pcg_update_restrict<2, true>) : go(k_pcg_update_restrict<2, false>);
}
void launch_pack_pcg(hipStream_t st, const LevelDev& L, const PcgDev& P) {
  if (L.nsub == 0) return;
  launch_kernel(k_pack_pcg, dim3(L.nsub), dim3(kNT), 0, st, L, P);
}
void launch_round_factors(hipStream_t st, const LevelDev& L, const PcgDev& P, int nrmax, int ncrmax, const double* Cr,
                          int* status) {
  if (P.prec == 0 || L.nsub == 0) return;
  const size_t lds = P.prec == 2 ? sizeof(double) * (2 * (size_t)nrmax * nrmax + 2 * (size_t)nrmax * ncrmax + nrmax) : 0;
  launch_kernel(k_round_factors, dim3(L.nsub), dim3(kNT), lds, st, L, P, nrmax, ncrmax, Cr, status);
}
void launch_pcg_prolong_post(hipStream_t st, const LevelDev& L, const PcgDev& P, int u) {
  if (P.nrhs > 1)
    launch_kernel(k_pcg_prolong_post<true>, dim3(P.nblk), dim3(kNT), 0, st, L, P, u);
  else
    launch_kernel(k_pcg_prolong_post<false>, dim3(P.nblk), dim3(kNT), 0, st, L, P, u);
}
void launch_build_phi(hipStream_t st, const LevelDev& L, int nif, const int32_t* sub_of_flat, const int32_t* phi_ptr,
                      int32_t* phi_ids, double* phi_w, const float* psi32) {
  if (nif == 0) return;
  launch_kernel(k_build_phi, dim3((nif + kNT - 1) / kNT), dim3(kNT), 0, st, L, nif, sub_of_flat, phi_ptr, phi_ids,
                phi_w, psi32);
}

}  // namespace bddc
