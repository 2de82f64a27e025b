// One deep level whose substructures are too large for one workgroup each
// (Algorithm "Multilevel BDDC" at level 2 with a direct coarsest solve), as
// four launches of many workgroups:
//   pre      r_2 gathered from the level-1 coarse contributions (ML-ri+1);
//            z_I = K_II^-1 r_I and t = K_GI K_II^-1 r_I (ML-uIi, ML-rBi) as
//            row blocks of dense products, several workgroups per substructure
//   restrict g = D (r_G - sum t), a = T_rr g_r, b = Psi^T g (k_apply_restrict)
//   coarse   r_3 = sum of b, u_3 = A_3^-1 r_3 (in every workgroup), and
//            v = D (a + Psi u_3) for every level-2 interface entry
//   post     u_B = sum over sharers of v (ML-uBi-1); u_I = z_I - K_II^-1 K_IG u_B
//            (ML-vIi, ML-ui), row blocks again
// Combining the interior pre- and post-corrections into z_I - M^T u_B with
// M = K_GI K_II^-1 = L_GI L^-1 removes the dependent triangular sweeps: every
// phase is a set of independent dense rows.
#include "dense.hpp"
#include "kernels.hpp"

namespace bddc {

// r_2 at level-2 dof k: the sum of the level-1 coarse contributions b1
__device__ inline double wide_r2(const WideDev& W, const double* b1, int k) {
  double acc = 0.0;
  for (int q = W.csh_ptr1[k]; q < W.csh_ptr1[k + 1]; ++q) acc += b1[W.csh_flat1[q]];
  return acc;
}

// r_2 = the sums of the level-1 coarse contributions, once for every column:
// at every level-2 dof (r2) and in the interior-flat order of the
// substructures (rIf); grid (blocks, columns)
__global__ void __launch_bounds__(kNT) k_wide_gather(WideDev W) {
  if (W.stop && *W.stop) return;
  const int c = blockIdx.y;
  const double* b1 = W.b1 + (size_t)c * W.ld_b1;
  for (int e = blockIdx.x * kNT + threadIdx.x; e < max(W.n2, W.nflat_i); e += gridDim.x * kNT) {
    if (e < W.n2) W.r2[(size_t)c * W.ld_r2 + e] = wide_r2(W, b1, e);
    if (e < W.nflat_i) W.rIf[(size_t)c * W.ld_i + e] = wide_r2(W, b1, W.L.int_gid[e]);
  }
}

// grid (chunks, substructures, column groups): rows [chunk*rows1, ...) of
// [K_II^-1 ; M] applied to the cols1 columns of the group (each operator row
// read once for all of them; a column's sums are those of a one-column launch)
__global__ void __launch_bounds__(kNT) k_wide_pre(WideDev W) {
  extern __shared__ double sh[];
  const LevelDev& L = W.L;
  const int s = blockIdx.y, chunk = blockIdx.x;
  if (s == L.nsub) {
    // the extra row: the r.r sums of the columns still iterating (the order
    // of block_sum_of, as the one-block sum launch forms them)
    __shared__ double red[kNT / 64];
    if (chunk != 0 || blockIdx.z != 0) return;
    for (int c = 0; c < W.nrhs; ++c) {
      if (W.sc[0].all_done || W.sc[c].done) continue;
      const double v = block_sum_of(W.rr_part + (size_t)c * W.rr_ld, W.rr_n, red);
      if (threadIdx.x == 0) W.sc[c].rrs = v;
    }
    return;
  }
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int r0 = chunk * W.rows1;
  if (r0 >= n) return;
  const int r1 = min(n, r0 + W.rows1);
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const double* Ki = W.Kinv + W.kioff[s];
  const double* Mt = W.Mt + W.moff[s];
  // one wave per row; rows < nI: column rho of the symmetric K_II^-1, else
  // column rho - nI of M^T (row of M): both contiguous.  Lane l takes the
  // entries l + 64 u (u < 4) of every 256; the first 256 of the wave's first
  // kAhead rows are loaded before r_2 is gathered (in-bounds clamped
  // addresses, entries past nI unused), so that gather hides their latency.
  auto column = [&](int rho) { return rho < nI ? Ki + (size_t)rho * nI : Mt + (size_t)(rho - nI) * nI; };
  auto load4 = [&](double (&cv)[4], const double* col, int jb) {
#pragma unroll
    for (int u = 0; u < 4; ++u) cv[u] = col[min(jb + lane + 64 * u, nI - 1)];
  };
  constexpr int kAhead = 2;
  double ahead[kAhead][4];
  if (nI > 0) {
#pragma unroll
    for (int q = 0; q < kAhead; ++q) load4(ahead[q], column(min(r0 + wave + 4 * q, r1 - 1)), 0);
  }
  if (W.stop && *W.stop) return;
  const int cb = blockIdx.z * W.cols1;            // first column of the group
  const int R = min(W.cols1, W.nrhs - cb);
  const double* b1 = W.b1 + (size_t)cb * W.ld_b1;
  double* r2 = W.r2 + (size_t)cb * W.ld_r2;
  double* Ly = L.y + (size_t)cb * W.ld_i;
  double* Lt = L.t + (size_t)cb * W.ld_g;
  double* rI = sh;   // column c at rI + c nI
  if (W.gathered) {
    // r_2 gathered by k_wide_gather: the substructure's interior entries
    const double* rIf = W.rIf + (size_t)cb * W.ld_i + L.ioff[s];
    for (int idx = tid; idx < R * nI; idx += kNT) {
      const int c = idx / nI, i = idx - c * nI;
      rI[idx] = rIf[(size_t)c * W.ld_i + i];
    }
  } else {
    for (int idx = tid; idx < R * nI; idx += kNT) {
      const int c = idx / nI, i = idx - c * nI;
      const int k = L.int_gid[L.ioff[s] + i];
      const double v = wide_r2(W, b1 + (size_t)c * W.ld_b1, k);
      rI[idx] = v;
      if (chunk == 0) r2[(size_t)c * W.ld_r2 + k] = v;
    }
  }
  if (chunk == 0 && !W.gathered)
    for (int idx = tid; idx < R * ng; idx += kNT) {
      const int c = idx / ng, a = idx - c * ng;
      const int k = L.gam_gid[L.goff[s] + a];
      r2[(size_t)c * W.ld_r2 + k] = wide_r2(W, b1 + (size_t)c * W.ld_b1, k);   // every sharer stores the same value
    }
  __syncthreads();
  for (int rho = r0 + wave, q = 0; rho < r1; rho += kNT / 64, ++q) {
    const double* col = column(rho);
    double acc[kMaxRhs][4];
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c) acc[c][0] = acc[c][1] = acc[c][2] = acc[c][3] = 0.0;
    auto terms = [&](const double (&cv)[4], int jb) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = jb + lane + 64 * u;
        if (j < nI) {
#pragma unroll
          for (int c = 0; c < kMaxRhs; ++c) {
            if (c >= R) break;
            acc[c][u] += cv[u] * rI[c * nI + j];
          }
        }
      }
    };
    if (nI > 0) {
      double cv[4];
      if (q < kAhead) {
#pragma unroll
        for (int t = 0; t < kAhead; ++t)
          if (q == t)
#pragma unroll
            for (int u = 0; u < 4; ++u) cv[u] = ahead[t][u];
      } else {
        load4(cv, col, 0);
      }
      terms(cv, 0);
      for (int jb = 256; jb < nI; jb += 256) {
        load4(cv, col, jb);
        terms(cv, jb);
      }
    }
#pragma unroll
    for (int c = 0; c < kMaxRhs; ++c) {
      if (c >= R) break;
      double v = (acc[c][0] + acc[c][1]) + (acc[c][2] + acc[c][3]);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      if (lane == 0) {
        if (rho < nI) Ly[(size_t)c * W.ld_i + L.ioff[s] + rho] = v;
        else Lt[(size_t)c * W.ld_g + L.goff[s] + rho - nI] = v;
      }
    }
  }
}

// the coarsest problem (solved by every workgroup when it is small; kInv: its
// solution u_3 already formed in W.u3 by the product with A_L^-1) and the
// prolongation of u_3 to the workgroup's slice of interface entries
// grid (blocks, columns)
template <bool kInv>
__global__ void __launch_bounds__(kNT) k_wide_coarse(WideDev W) {
  constexpr int kCK = 8;   // coarse dofs per substructure held in registers
  extern __shared__ double sh[];
  const LevelDev& L = W.L;
  const int col = blockIdx.y;
  const double* La = L.a + (size_t)col * W.ld_g;
  double* Lv = L.v + (size_t)col * W.ld_g;
  // the operands of the thread's first interface entry (its row of Psi, the
  // coarse ids, a and delta), loaded before the coarsest problem is solved
  const int f0 = blockIdx.x * kNT + threadIdx.x;
  int a0 = 0, ng0 = 0, c00 = 0, ncs0 = 0;
  const double* P0 = nullptr;
  double pv[kCK], la0 = 0.0, dl0 = 0.0;
  int cv[kCK];
  if (f0 < W.nflat) {
    const int s = W.sub_of_flat[f0];
    a0 = f0 - L.goff[s];
    ng0 = (L.loc_ptr[s + 1] - L.loc_ptr[s]) - L.nint[s];
    c00 = L.coff[s];
    ncs0 = L.coff[s + 1] - c00;
    P0 = L.Psi + L.psioff[s];
    if (ncs0 > 0) {
#pragma unroll
      for (int k = 0; k < kCK; ++k) {
        const int kk = min(k, ncs0 - 1);
        pv[k] = P0[a0 + (size_t)kk * ng0];
        cv[k] = L.cid[c00 + kk];
      }
    }
    la0 = La[f0];
    dl0 = L.delta[f0];
  }
  if (W.stop && *W.stop) return;
  const double* u3;
  if constexpr (kInv) {
    u3 = W.u3 + (size_t)col * W.ld_3;
  } else {
    const double* Lb = L.b + (size_t)col * W.ld_c;
    double* y = sh;
    for (int k = threadIdx.x; k < W.ncL; k += kNT) {
      double acc = 0.0;
      for (int q = L.csh_ptr[k]; q < L.csh_ptr[k + 1]; ++q) acc += Lb[L.csh_flat[q]];
      y[k] = acc;
    }
    __syncthreads();
    wg_trsv_lower(W.AL, W.ncL, W.ncL, y);
    wg_trsv_lower_trans(W.AL, W.ncL, W.ncL, y);
    u3 = y;
  }
  if (f0 < W.nflat) {
    double w = la0;
#pragma unroll
    for (int k = 0; k < kCK; ++k)
      if (k < ncs0) w += pv[k] * u3[cv[k]];
    for (int k0 = kCK; k0 < ncs0; k0 += kCK) {   // the rest: kCK loads in flight
#pragma unroll
      for (int k = 0; k < kCK; ++k) {
        const int kk = min(k0 + k, ncs0 - 1);
        pv[k] = P0[a0 + (size_t)kk * ng0];
        cv[k] = L.cid[c00 + kk];
      }
#pragma unroll
      for (int k = 0; k < kCK; ++k)
        if (k0 + k < ncs0) w += pv[k] * u3[cv[k]];
    }
    Lv[f0] = dl0 * w;
  }
  for (int f = f0 + gridDim.x * kNT; f < W.nflat; f += gridDim.x * kNT) {
    const int s = W.sub_of_flat[f];
    const int a = f - L.goff[s];
    const int ng = (L.loc_ptr[s + 1] - L.loc_ptr[s]) - L.nint[s];
    const int c0 = L.coff[s], ncs = L.coff[s + 1] - c0;
    const double* P = L.Psi + L.psioff[s];
    double w = La[f];
    for (int k = 0; k < ncs; ++k) w += P[a + (size_t)k * ng] * u3[L.cid[c0 + k]];
    Lv[f] = L.delta[f] * w;
  }
}

// grid (chunks of 64 interior rows, substructures, columns): u_B, then
// u_I = z_I - M^T u_B with four threads per row (fixed-order reduction).
// Thread (row, a0) holds its first kPostK entries of M^T (columns a0,
// a0 + 4, ...) and z_I, loaded before u_B is gathered.
__global__ void __launch_bounds__(kNT) k_wide_post(WideDev W) {
  constexpr int kPostK = 24;
  extern __shared__ double sh[];
  const LevelDev& L = W.L;
  const int s = blockIdx.y, chunk = blockIdx.x, col = blockIdx.z;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int g0 = L.goff[s];
  const int tid = threadIdx.x;
  if (chunk * 64 >= max(nI, 1)) return;
  const int il = tid & 63, ag = tid >> 6;
  const int i = chunk * 64 + il;
  const double* Mt = W.Mt + W.moff[s];
  const double* Ly = L.y + (size_t)col * W.ld_i;
  double mv[kPostK];
  double zi = 0.0;
  if (nI > 0) {
    const int ic = min(i, nI - 1);
    if (ng > 0) {
#pragma unroll
      for (int k = 0; k < kPostK; ++k) mv[k] = Mt[ic + (size_t)min(ag + 4 * k, ng - 1) * nI];
    }
    zi = Ly[L.ioff[s] + ic];
  }
  if (W.stop && *W.stop) return;
  const double* Lv = L.v + (size_t)col * W.ld_g;
  double* u2 = W.u2 + (size_t)col * W.ld_u2;
  double* uB = sh;
  double* part = sh + ng;
  for (int a = tid; a < ng; a += kNT) {
    const int f = g0 + a;
    const int gi = L.gam_iid[f];
    double acc = 0.0;
    for (int k = L.sh_ptr[gi]; k < L.sh_ptr[gi + 1]; ++k) acc += Lv[L.sh_flat[k]];
    uB[a] = acc;
    if (chunk == 0 && L.sh_flat[L.sh_ptr[gi]] == f) u2[L.gam_gid[f]] = acc;
  }
  __syncthreads();
  double acc = 0.0;
  if (i < nI) {
#pragma unroll
    for (int k = 0; k < kPostK; ++k)
      if (ag + 4 * k < ng) acc += mv[k] * uB[ag + 4 * k];
    for (int a0 = ag + 4 * kPostK; a0 < ng; a0 += 32) {   // the rest: eight loads in flight
      double m8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) m8[u] = Mt[i + (size_t)min(a0 + 4 * u, ng - 1) * nI];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (a0 + 4 * u < ng) acc += m8[u] * uB[a0 + 4 * u];
    }
  }
  part[tid] = acc;
  __syncthreads();
  if (ag == 0 && i < nI) {
    const double m = (part[il] + part[il + 64]) + (part[il + 128] + part[il + 192]);
    u2[L.int_gid[L.ioff[s] + i]] = zi - m;
  }
}

// setup: K_II^-1 = L^-T L^-1 and M^T = L^-T L_GI^T from the explicit L^-1
// (column-major, lower) and the factored K (L_GI in rows nI.. of the first nI
// columns); one thread per entry, grid (blocks, substructures)
__global__ void __launch_bounds__(kNT) k_wide_ops(LevelDev L, double* __restrict__ Kinv,
                                                  const int64_t* __restrict__ kioff, double* __restrict__ Mt,
                                                  const int64_t* __restrict__ moff) {
  const int s = blockIdx.y;
  const int n = L.loc_ptr[s + 1] - L.loc_ptr[s];
  const int nI = L.nint[s];
  const int ng = n - nI;
  const int e = blockIdx.x * kNT + threadIdx.x;
  const double* Li = L.Linv + L.linvoff[s];
  const double* A = L.K + L.koff[s];
  if (e < nI * nI) {
    const int i = e % nI, j = e / nI;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int p = max(i, j);
    for (; p + 3 < nI; p += 4) {
      acc[0] += Li[p + (size_t)i * nI] * Li[p + (size_t)j * nI];
      acc[1] += Li[p + 1 + (size_t)i * nI] * Li[p + 1 + (size_t)j * nI];
      acc[2] += Li[p + 2 + (size_t)i * nI] * Li[p + 2 + (size_t)j * nI];
      acc[3] += Li[p + 3 + (size_t)i * nI] * Li[p + 3 + (size_t)j * nI];
    }
    for (; p < nI; ++p) acc[0] += Li[p + (size_t)i * nI] * Li[p + (size_t)j * nI];
    Kinv[kioff[s] + e] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  } else if (e < nI * nI + nI * ng) {
    const int e2 = e - nI * nI;
    const int j = e2 % nI, a = e2 / nI;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int p = j;
    for (; p + 3 < nI; p += 4) {
      acc[0] += A[(nI + a) + (size_t)p * n] * Li[p + (size_t)j * nI];
      acc[1] += A[(nI + a) + (size_t)(p + 1) * n] * Li[p + 1 + (size_t)j * nI];
      acc[2] += A[(nI + a) + (size_t)(p + 2) * n] * Li[p + 2 + (size_t)j * nI];
      acc[3] += A[(nI + a) + (size_t)(p + 3) * n] * Li[p + 3 + (size_t)j * nI];
    }
    for (; p < nI; ++p) acc[0] += A[(nI + a) + (size_t)p * n] * Li[p + (size_t)j * nI];
    Mt[moff[s] + e2] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  }
}

void launch_wide_ops(hipStream_t st, const LevelDev& L, int nmax_ops, double* Kinv, const int64_t* kioff, double* Mt,
                     const int64_t* moff) {
  if (L.nsub == 0 || nmax_ops == 0) return;
  launch_kernel(k_wide_ops, dim3((nmax_ops + kNT - 1) / kNT, L.nsub), dim3(kNT), 0, st, L, Kinv, kioff, Mt, moff);
}

void launch_wide_pre(hipStream_t st, const WideDev& W) {
  if (W.nrhs < 1 || W.nrhs > kMaxRhs) throw std::invalid_argument("launch_wide_pre: bad column count");
  // several columns: a small grid (< 1024 workgroups per column) keeps one
  // grid slice per column; a large one takes every column in each workgroup,
  // with up to four times the rows while the grid keeps >= 1024 workgroups,
  // so fewer workgroups gather the same r_I
  WideDev V = W;
  const int wgs = W.nchunk1 * W.L.nsub;
  V.cols1 = wgs < 1024 ? 1 : W.nrhs;
  if (V.cols1 > 1) {
    const int f = std::min(4, std::max(1, wgs / 1024));
    V.rows1 = W.rows1 * f;
    V.nchunk1 = (W.nchunk1 + f - 1) / f;
  }
  // several columns: r_2 gathered once, not by every workgroup
  V.gathered = W.nrhs > 1 ? 1 : 0;
  if (V.gathered) {
    const int nb = std::max(1, std::min(1024, (std::max(W.n2, W.nflat_i) + kNT - 1) / kNT));
    launch_kernel(k_wide_gather, dim3(nb, W.nrhs), dim3(kNT), 0, st, V);
  }
  const int groups = (W.nrhs + V.cols1 - 1) / V.cols1;
  launch_kernel(k_wide_pre, dim3(V.nchunk1, V.L.nsub + (V.sc ? 1 : 0), groups), dim3(kNT),
                sizeof(double) * (size_t)V.cols1 * max(V.nImax, 1), st, V);
}

void launch_wide_coarse(hipStream_t st, const WideDev& W) {
  if (W.coarse_inv) {
    launch_coarse_gather_cols(st, W.ncL, W.L.csh_ptr, W.L.csh_flat, W.L.b, W.ld_c, W.r3, W.ld_3, W.nrhs, W.stop);
    launch_coarse_inv_apply(st, W.ncL, W.AL, W.r3, W.ld_3, W.u3, W.ld_3, W.nrhs, W.stop);
    const int nb = max(1, (W.nflat + kNT - 1) / kNT);
    launch_kernel(k_wide_coarse<true>, dim3(nb, W.nrhs), dim3(kNT), 0, st, W);
    return;
  }
  const int nb = max(1, min(64, (W.nflat + kNT - 1) / kNT));
  launch_kernel(k_wide_coarse<false>, dim3(nb, W.nrhs), dim3(kNT), sizeof(double) * (size_t)max(W.ncL, 1), st, W);
}

void launch_wide_post(hipStream_t st, const WideDev& W) {
  launch_kernel(k_wide_post, dim3(W.nchunk4, W.L.nsub, W.nrhs), dim3(kNT), sizeof(double) * ((size_t)W.ngmax + kNT),
                st, W);
}

}  // namespace bddc
