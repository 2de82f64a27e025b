// Deep level and coarsest solve of Algorithm "Multilevel BDDC" (Section 2.1)
// in one cooperative launch, for hierarchies with one level between the
// level-1 interface problem and the coarsest direct solve.
//
// One workgroup per level-2 substructure.  Its operators (interior factor
// inverse, L_GI, T_rr, Psi, stiffness weights) and index lists are packed at
// setup into one contiguous block each, so the prefetch into LDS at the start
// is a single coalesced copy.  Two grid barriers separate the phases that read
// other substructures' results:
//   1. after the interior corrections t (the restriction sums t over sharers);
//   2. after the restriction (the coarse right-hand side sums b over sharers).
// Every workgroup then solves the small coarsest problem redundantly with the
// explicit inverse of its Cholesky factor.  The interface average of the
// prolongation, u_B = sum_s delta_s (T_rr g_s + Psi_s u_c) over the sharers,
// is split as sum_s delta_s T_rr g_s (published before barrier 2) plus a row
// of the delta-weighted coarse basis of all sharers (packed at setup) times
// u_c, so no barrier is needed after the coarse solve.
#include <string>

#include "common.hpp"
#include "dense.hpp"
#include "kernels.hpp"

namespace bddc {

namespace {

constexpr int kSpinLimit = 1 << 22;   // about 0.1 s of polling; past it the status flags a failure

// Grid barrier without cache maintenance.  Every value one workgroup hands
// to another across a barrier (t, then da and b) is written and read with
// agent-scope atomic accesses, which are coherent across the XCDs' L2
// caches; so the barrier only has to order them: each thread's stores have
// completed (s_waitcnt) before the workgroup arrives, and the reads after it
// are issued once every workgroup has arrived.  A release / acquire pair at
// agent scope would instead write back and invalidate the L2 of every XCD
// at every barrier (measured: 4.0 and 4.7 us per barrier, 16 workgroups).
// The arrival counter only grows (reset before each solve): barrier k of the
// launch completes when it reaches (done + k + 1) x nblocks, where `done`
// (thread 0's `passed`) counts the barriers completed before; no workgroup
// can complete one before all have arrived, so the count read at the start
// of the launch, divided by nblocks, gives it.  The spin is bounded; past
// the bound the status flags a failure.
__device__ void grid_barrier(unsigned* count, unsigned nblocks, int* status, unsigned& passed) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned target = (passed + 1) * nblocks;
    if (__hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 != target) {
      int spins = 0;
      while (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > kSpinLimit) {
          atomicOr(status, 4);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    ++passed;
  }
  __syncthreads();
}

// values handed between workgroups across a grid barrier
__device__ inline void xstore(double* p, double v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline double xload(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// out(c, i) = sum_{j in [j0(i), j1(i))} A[i*rs + j*cs] x_c[j] for i < rows and
// the R columns x_c = x + c * xs, eight lanes per row (fixed reduction order),
// then store(c, i, value) on lane 0 of the eight: row t of the combined loop
// is row i = t mod rows of column c = t / rows.  With xi, x_c is read at
// xi[j] (a gathered product).
// (kMulti false: the one column 0, no index division)
template <bool kMulti, class J0, class J1, class Store>
__device__ inline void mv8c(int rows, int R, const double* A, int rs, int cs, const double* x, int xs, J0 j0f,
                            J1 j1f, Store store, const int32_t* xi = nullptr) {
  const int sub = threadIdx.x & 7;
  const int tot = kMulti ? rows * R : rows;
  for (int t = threadIdx.x >> 3; t < tot; t += kCoopNT / 8) {
    const int c = kMulti ? t / rows : 0, i = kMulti ? t - c * rows : t;
    const double* xc = x + (size_t)c * xs;
    double acc = 0.0;
    const int j1 = j1f(i);
    for (int j = j0f(i) + sub; j < j1; j += 8) acc += A[(size_t)i * rs + (size_t)j * cs] * xc[xi ? xi[j] : j];
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 4);
    if (sub == 0) store(c, i, acc);
  }
}

template <class T>
__device__ inline void copy_batched(T* dst, const T* __restrict__ src, int n) {
  for (int base = threadIdx.x; base < n; base += 8 * kCoopNT) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (base + u * kCoopNT < n) ? src[base + u * kCoopNT] : T(0);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (base + u * kCoopNT < n) dst[base + u * kCoopNT] = v[u];
  }
}

}  // namespace

template <bool kMulti>
__global__ void __launch_bounds__(kCoopNT) k_deep_coop(CoopDev C) {
  if (C.stop && *C.stop) return;
  extern __shared__ double sh[];
  const int s = blockIdx.x, tid = threadIdx.x;
  // grid barriers completed before this launch
  unsigned passed = tid == 0 ? __hip_atomic_load(C.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) / gridDim.x : 0u;
  const int32_t* me = C.meta + (size_t)kCoopMeta * s;
  const int nI = me[0], ng = me[1], nr = me[2], ncs = me[3], nsh = me[4], ng1 = me[5], goff = me[6], coff = me[7];
  const int n = nI + ng;
  const int ncL = C.ncL;
  const int R = kMulti ? C.nrhs : 1;     // columns: vectors below hold R columns each
  const int mI = C.nImax, mG = C.ngmax;  // their column strides
  (void)me[8];
  // LDS: operator block | vectors | coarsest inverse factor | ints
  double* Li = sh;                                   // K_II^-1, nI x nI
  double* G = Li + (size_t)nI * nI;                  // M^T = (K_GI K_II^-1)^T, nI x ng
  double* Tm = G + (size_t)ng * nI;                  // nr x nr
  double* Ps = Tm + (size_t)nr * nr;                 // ng x ncs
  double* dl = Ps + (size_t)ng * ncs;                // ng
  double* phw = dl + ng;                             // phi weights
  double* rI = sh + C.opmax;                         // R x nImax
  double* rG = rI + (size_t)R * mI;                  // R x ngmax
  double* y = rG + (size_t)R * mG;                   // R x nImax
  double* g = y + (size_t)R * mI;                    // R x ngmax
  double* av = g + (size_t)R * mG;                   // R x ngmax
  double* uB = av + (size_t)R * mG;                  // R x ngmax
  double* LL = uB + (size_t)R * mG;
  double* rc = LL + (size_t)ncL * ncL;               // R x ncL
  double* wc = rc + (size_t)R * ncL;                 // R x ncL
  double* uc = wc + (size_t)R * ncL;                 // R x ncL
  int32_t* ib = reinterpret_cast<int32_t*>(uc + (size_t)R * ncL);
  int32_t* int_gid = ib;
  int32_t* gam_gid = int_gid + nI;
  int32_t* own = gam_gid + ng;
  int32_t* shp = own + ng;
  int32_t* shf = shp + ng + 1;
  int32_t* gp = shf + nsh;
  int32_t* gf = gp + n + 1;
  int32_t* cid = gf + ng1;
  int32_t* phi_ptr = cid + ncs;
  int32_t* phi_ids = phi_ptr + ng + 1;
  int32_t* cg = ib + C.idxmax;
  (void)cid;

  // prefetch: operators + coarsest factor inverse, and index lists + coarse
  // gather, with every load of the first kPD / kPI per thread issued before
  // any store (one round of memory latency); larger blocks finish in a loop
  {
    const double* opg = C.ops + C.opoff[s];
    const int nop = (int)(C.opoff[s + 1] - C.opoff[s]), nll = ncL * ncL;
    const int32_t* ixg = C.idx + C.idxoff[s];
    const int nix = (int)(C.idxoff[s + 1] - C.idxoff[s]), ncg = C.cg_len;
    constexpr int kPD = 24, kPI = 8;
    double vd[kPD];
    int32_t vi[kPI];
#pragma unroll
    for (int u = 0; u < kPD; ++u) {
      const int v = tid + u * kCoopNT;
      vd[u] = v < nop ? opg[v] : (v < nop + nll ? C.LLinv[v - nop] : 0.0);
    }
#pragma unroll
    for (int u = 0; u < kPI; ++u) {
      const int v = tid + u * kCoopNT;
      vi[u] = v < nix ? ixg[v] : (v < nix + ncg ? C.cg[v - nix] : 0);
    }
#pragma unroll
    for (int u = 0; u < kPD; ++u) {
      const int v = tid + u * kCoopNT;
      if (v < nop) sh[v] = vd[u];
      else if (v < nop + nll) LL[v - nop] = vd[u];
    }
#pragma unroll
    for (int u = 0; u < kPI; ++u) {
      const int v = tid + u * kCoopNT;
      if (v < nix) ib[v] = vi[u];
      else if (v < nix + ncg) cg[v - nix] = vi[u];
    }
    const int d0 = kPD * kCoopNT, i0 = kPI * kCoopNT;
    if (nop > d0) copy_batched(sh + d0, opg + d0, nop - d0);
    if (nop + nll > d0) {
      const int l0 = d0 > nop ? d0 - nop : 0;
      copy_batched(LL + l0, C.LLinv + l0, nll - l0);
    }
    if (nix > i0) copy_batched(ib + i0, ixg + i0, nix - i0);
    if (nix + ncg > i0) {
      const int c0 = i0 > nix ? i0 - nix : 0;
      copy_batched(cg + c0, C.cg + c0, ncg - c0);
    }
  }
  __syncthreads();
  // Every phase below runs for all R columns before the next barrier (column
  // c of a global vector at c times its stride), so R columns cost the
  // barriers of one.
  // r_2 on the local dofs: sums of the level-1 coarse contributions
  for (int t = tid; t < n * R; t += kCoopNT) {
    const int c = kMulti ? t / n : 0, p = kMulti ? t - c * n : t;
    const double* b1 = C.b1 + (size_t)c * C.ld_b1;
    double acc = 0.0;
    for (int q = gp[p]; q < gp[p + 1]; ++q) acc += b1[gf[q]];
    if (p < nI) rI[c * mI + p] = acc;
    else rG[c * mG + p - nI] = acc;
  }
  __syncthreads();
  // interior correction (ML-uIi, ML-rBi): y = K_II^-1 r_I and t = K_GI K_II^-1 r_I
  // in one pass: row rho of [K_II^-1 ; M] is column rho of [K_II^-1  M^T]
  mv8c<kMulti>(nI + ng, R, Li, nI, 1, rI, mI, [](int) { return 0; }, [&](int) { return nI; },
       [&](int c, int i, double v) {
         if (i < nI) y[c * mI + i] = v;
         else xstore(&C.t[(size_t)c * C.ld_t + goff + i - nI], v);
       });
  grid_barrier(C.bar, gridDim.x, C.status, passed);
  // g = delta (r_G - sum t);  a = T_rr g_r (ML-wDi);  b = Psi^T g (ML-coarse)
  for (int t = tid; t < ng * R; t += kCoopNT) {
    const int c = kMulti ? t / ng : 0, a = kMulti ? t - c * ng : t;
    const double* tc = C.t + (size_t)c * C.ld_t;
    double v = rG[c * mG + a];
    for (int q = shp[a]; q < shp[a + 1]; ++q) v -= xload(&tc[shf[q]]);
    g[c * mG + a] = dl[a] * v;
  }
  __syncthreads();
  mv8c<kMulti>(nr, R, Tm, 1, nr, g, mG, [](int) { return 0; }, [&](int) { return nr; },
       [&](int c, int a, double v) { xstore(&C.da[(size_t)c * C.ld_t + goff + a], dl[a] * v); });
  for (int t = tid; t < (ng - nr) * R; t += kCoopNT) {
    const int c = kMulti ? t / (ng - nr) : 0, a = nr + (kMulti ? t - c * (ng - nr) : t);
    xstore(&C.da[(size_t)c * C.ld_t + goff + a], 0.0);
  }
  mv8c<kMulti>(ncs, R, Ps, ng, 1, g, mG, [](int) { return 0; }, [&](int) { return ng; },
       [&](int c, int k, double v) { xstore(&C.b[(size_t)c * C.ld_b + coff + k], v); });
  grid_barrier(C.bar, gridDim.x, C.status, passed);
  // coarsest right-hand side r_c = sum of the coarse contributions, and the
  // sharers' sum of delta T_rr g on the interface, in one round of loads
  for (int t = tid; t < ncL * R; t += kCoopNT) {
    const int c = kMulti ? t / ncL : 0, k = kMulti ? t - c * ncL : t;
    const double* bc = C.b + (size_t)c * C.ld_b;
    double acc = 0.0;
    for (int q = cg[k]; q < cg[k + 1]; ++q) acc += xload(&bc[cg[ncL + 1 + q]]);
    rc[c * ncL + k] = acc;
  }
  for (int t = tid; t < ng * R; t += kCoopNT) {
    const int c = kMulti ? t / ng : 0, a = kMulti ? t - c * ng : t;
    const double* dc = C.da + (size_t)c * C.ld_t;
    double acc = 0.0;
    for (int q = shp[a]; q < shp[a + 1]; ++q) acc += xload(&dc[shf[q]]);
    av[c * mG + a] = acc;
  }
  __syncthreads();
  mv8c<kMulti>(ncL, R, LL, 1, ncL, rc, ncL, [](int) { return 0; }, [](int i) { return i + 1; },
       [&](int c, int i, double v) { wc[c * ncL + i] = v; });
  __syncthreads();
  mv8c<kMulti>(ncL, R, LL, ncL, 1, wc, ncL, [](int i) { return i; }, [&](int) { return ncL; },
       [&](int c, int i, double v) { uc[c * ncL + i] = v; });
  __syncthreads();
  // u_B = sum over sharers of delta (T_rr g + Psi u_c)   (ML-uBi-1), owner writes
  mv8c<kMulti>(ng, R, phw, 0, 1, uc, ncL, [&](int a) { return phi_ptr[a]; }, [&](int a) { return phi_ptr[a + 1]; },
       [&](int c, int a, double v) {
         const double u = av[c * mG + a] + v;
         uB[c * mG + a] = u;
         if (own[a]) C.u2[(size_t)c * C.ld_u2 + gam_gid[a]] = u;
       },
       phi_ids);
  __syncthreads();
  // u_I = K_II^-1 (r_I - K_IG u_B) = y - M^T u_B   (ML-vIi, ML-ui)
  mv8c<kMulti>(nI, R, G, 1, nI, uB, mG, [](int) { return 0; }, [&](int) { return ng; },
       [&](int c, int i, double v) { C.u2[(size_t)c * C.ld_u2 + int_gid[i]] = y[c * mI + i] - v; });
}

size_t coop_lds(const CoopDev& C) {
  const size_t R = (size_t)std::max(1, C.nrhs);
  const size_t dbl = (size_t)C.opmax + R * (2 * (size_t)C.nImax + 4 * (size_t)C.ngmax + 3 * (size_t)C.ncL) +
                     (size_t)C.ncL * C.ncL;
  return sizeof(double) * dbl + sizeof(int32_t) * ((size_t)C.idxmax + C.cg_len);
}

int coop_max_blocks(size_t lds) {
  int dev = 0, ncu = 0, per = 0, coop = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_deep_coop<true>, kCoopNT, lds) != hipSuccess) return 0;
  return per * ncu;
}

// The grid barriers need every workgroup resident.  The grid is at most the
// device's cooperative capacity (checked when the path is chosen).  While the
// process holds a single handle, the launch follows the previous kernel of
// the same stream and nothing else of the library runs beside it, so an
// ordinary launch finds room for every workgroup; with several live handles
// (other streams may hold the compute units) the caller asks for the
// cooperative API, which guarantees residency at about 25 us of queue
// synchronisation per launch (also forced by BDDC_COOP_LAUNCH=1).  If
// residency ever failed, the bounded spin ends the kernel and the status flag
// reports it; the next solve resets the barrier (launch_coop_reset).
void launch_deep_coop(hipStream_t st, const CoopDev& C, bool cooperative) {
  if (!cooperative) {
    if (C.nrhs > 1)
      launch_kernel(k_deep_coop<true>, dim3(C.nsub), dim3(kCoopNT), coop_lds(C), st, C);
    else
      launch_kernel(k_deep_coop<false>, dim3(C.nsub), dim3(kCoopNT), coop_lds(C), st, C);
    return;
  }
  // a cooperative launch takes no dispatch events: record them around it instead
  const LaunchEvents ev = g_launch_events;
  g_launch_events = LaunchEvents{};
  if (ev.start) (void)hipEventRecord(ev.start, st);
  CoopDev arg = C;
  void* args[] = {&arg};
  const void* kern = C.nrhs > 1 ? reinterpret_cast<const void*>(k_deep_coop<true>)
                                 : reinterpret_cast<const void*>(k_deep_coop<false>);
  const hipError_t e = hipLaunchCooperativeKernel(kern, dim3(C.nsub),
                                                  dim3(kCoopNT), args, coop_lds(C), st);
  if (e != hipSuccess) fail(BDDC_EDEVICE, std::string("cooperative launch: ") + hipGetErrorString(e));
  if (ev.stop) (void)hipEventRecord(ev.stop, st);
}

// Barrier counter, generation and the barrier-timeout status bit back to
// zero before a solve: a timed-out barrier leaves the counter mid-way, and
// every later launch must start from a clean state.  A kernel, not a memset,
// so that the reset can sit in a captured stream.
__global__ void k_coop_reset(unsigned* bar, int* status) {
  if (threadIdx.x == 0) {
    bar[0] = 0u;
    bar[1] = 0u;
    *status &= ~4;
  }
}

void launch_coop_reset(hipStream_t st, const CoopDev& C) {
  launch_kernel(k_coop_reset, dim3(1), dim3(64), 0, st, C.bar, C.status);
}

// pack the level-2 operators of one substructure per workgroup
__global__ void __launch_bounds__(kNT) k_pack_coop(LevelDev L, CoopDev C) {
  const int s = blockIdx.x;
  const int32_t* me = C.meta + (size_t)kCoopMeta * s;
  const int nI = me[0], ng = me[1], nr = me[2], ncs = me[3];
  const int n = nI + ng;
  double* o = const_cast<double*>(C.ops) + C.opoff[s];
  const double* Ki = C.Kinv + C.kioff[s];
  const double* Mt = C.Mt + C.moff[s];
  const double* T = L.T + L.toff[s];
  const double* P = L.Psi + L.psioff[s];
  for (int idx = threadIdx.x; idx < nI * nI; idx += kNT) o[idx] = Ki[idx];
  o += (size_t)nI * nI;
  for (int idx = threadIdx.x; idx < nI * ng; idx += kNT) o[idx] = Mt[idx];
  o += (size_t)ng * nI;
  for (int idx = threadIdx.x; idx < nr * nr; idx += kNT) o[idx] = T[idx];
  o += (size_t)nr * nr;
  for (int idx = threadIdx.x; idx < ng * ncs; idx += kNT) o[idx] = P[idx];
  o += (size_t)ng * ncs;
  for (int a = threadIdx.x; a < ng; a += kNT) o[a] = L.delta[L.goff[s] + a];
  o += ng;
  // phi rows: for each interface dof, delta_{s'} Psi_{s'} row of every sharer s'
  const int32_t* ib = C.idx + C.idxoff[s];
  const int nsh = me[4], ng1 = me[5];
  const int32_t* shp = ib + nI + 2 * ng;
  const int32_t* shf = shp + ng + 1;
  const int32_t* phi_ptr = shf + nsh + (n + 1) + ng1 + ncs;
  for (int a = threadIdx.x; a < ng; a += kNT) {
    int j = phi_ptr[a];
    for (int q = shp[a]; q < shp[a + 1]; ++q) {
      const int f = shf[q];
      const int t = C.sub_of_flat[f];
      const int at = f - L.goff[t];
      const int ngt = (L.loc_ptr[t + 1] - L.loc_ptr[t]) - L.nint[t];
      const int ncst = L.coff[t + 1] - L.coff[t];
      const double* Pt = L.Psi + L.psioff[t];
      for (int k = 0; k < ncst; ++k) o[j++] = L.delta[f] * Pt[at + (size_t)k * ngt];
    }
  }
}

void launch_pack_coop(hipStream_t st, const LevelDev& L, const CoopDev& C) {
  launch_kernel(k_pack_coop, dim3(C.nsub), dim3(kNT), 0, st, L, C);
}

// X = L^{-1} for one dense lower-triangular matrix (ld ld, order m), by the
// in-place Gauss-Jordan steps of the interior triangular inverse, in LDS
__global__ void __launch_bounds__(kNT) k_tri_inverse_dense(const double* __restrict__ L, int ld, int m,
                                                           double* __restrict__ X) {
  extern __shared__ double sh[];
  double* M = sh;
  double* rowk = M + (size_t)m * m;
  double* colk = rowk + m;
  const int tid = threadIdx.x;
  for (ColWalk w_(tid, kNT, m); w_.j < m; w_.next()) {
    const int i = w_.i, j = w_.j;
    [[maybe_unused]] const int idx = i + j * m;
    M[idx] = (i >= j) ? L[i + (size_t)j * ld] : 0.0;
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
  for (int idx = tid; idx < m * m; idx += kNT) X[idx] = M[idx];
}

void launch_tri_inverse_dense(hipStream_t st, const double* L, int ld, int m, double* X) {
  if (m <= 0) return;
  launch_kernel(k_tri_inverse_dense, dim3(1), dim3(kNT), sizeof(double) * ((size_t)m * m + 2 * (size_t)m), st, L,
                ld, m, X);
}

}  // namespace bddc
