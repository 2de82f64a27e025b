// The two operator-streaming launches of the PCG iteration on the level-1
// interface (Section 5; the product with the local Schur complements and the
// restriction with the substructure correction of Algorithm "Multilevel
// BDDC", Section 2.1) for wide interfaces: substructures whose interfaces
// hold hundreds of dofs (uneven regions of thousands of local dofs).
//
// One workgroup per substructure leaves too few loads in flight there: a
// 400 x 400 S_s read by one thread per row keeps each thread on one long
// chain of dependent batches.  Here the rows of S_s (and of T_rr) are cut
// into blocks of 64 and every block gets a workgroup of four waves; wave w
// reads the columns of its quarter, lane l row 64 rb + l, so every load is
// 64 consecutive entries of one column (full column-major storage, columns
// starting on 128-byte boundaries), sixteen loads in flight per lane, and each entry is applied to every live
// right-hand side.  The wave partials are summed in wave order, so a column
// solved alone and the same column in a blocked solve give bitwise the same
// result.  The vectors a block needs (p_s, or g = delta r_s) are gathered by
// every block of the substructure; the blocks of one substructure are laid
// out so that they run on one XCD (workgroups are dealt to the eight XCDs in
// turn), where the second gather hits that XCD's L2.
//
// Scalars (alpha, beta) come from the one-block sums (PcgDev::fin); the
// energies p_s^T S_s p_s are left per row block (PcgDev::npq partials).
#include "dense.hpp"
#include "kernels.hpp"

namespace bddc {

namespace {

constexpr int kRows = 64;   // rows of a block (one per lane)
constexpr int kBatch = 16;  // loads in flight per lane
constexpr int kRT = 256;    // threads of a block's workgroup
constexpr int kNW = kRT / 64;

// workgroup -> (substructure, row block): groups of eight substructures take
// 8 * nrb consecutive workgroups, block rb of substructure 8 G + j at
// 8 (G nrb + rb) + j, so all blocks of a substructure share b mod 8
__device__ inline void row_task(int nrb, int& s, int& rb) {
  const int b = blockIdx.x;
  const int grp = b / (8 * nrb), w = b - grp * 8 * nrb;
  rb = w >> 3;
  s = grp * 8 + (w & 7);
}

// acc[k] += sum over columns j in [j0, j1) of A[row, j] v[j][k]: A column-major
// (leading dimension ld, already offset to the row), v in LDS as [j][k] with
// stride kNL.  All kNL accumulators run (entries of columns past the live
// ones are zero in v): no branch in the loop, and each column's sum is the
// same whatever the other columns hold
// (the last batch loads at clamped column indices and adds zero terms past
// j1, so a ragged end costs one batch, not a chain of single loads)
// A is the block's first row (the same for the whole wave) and `row` the
// lane's row in it, so every load takes a wave-uniform column address plus
// a 32-bit lane offset (one register for the lane part of all the loads).
template <int kNL, class T>
__device__ inline void row_product(double (&acc)[kNL], const T* __restrict__ A, int row, int ld, int j0, int j1,
                                   const double* v) {
  for (int j = j0; j < j1; j += kBatch) {
    T t[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) t[q] = (A + (size_t)min(j + q, j1 - 1) * ld)[row];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      // past j1: a zero term on the last column (a select, so that the
      // loads above stay unconditional)
      const double a = j + q < j1 ? static_cast<double>(t[q]) : 0.0;
      const double* vj = v + (size_t)min(j + q, j1 - 1) * kNL;
      if constexpr (kNL == 1) {
        acc[0] += a * vj[0];
      } else {
#pragma unroll
        for (int k = 0; k < kNL; k += 2) {
          const double2 pv = *reinterpret_cast<const double2*>(vj + k);
          acc[k] += a * pv.x;
          acc[k + 1] += a * pv.y;
        }
      }
    }
  }
}

// live columns of the blocked solve into lc (same list on every thread)
__device__ inline int live_columns(const PcgDev& P, int* lc) {
  int nl = 0;
  for (int c = 0; c < P.nrhs; ++c)
    if (!P.sc[c].done) lc[nl++] = c;
  return nl;
}

}  // namespace

// p_k = z + beta p_{k-1} (owners store p_k), q_s = S_s p_s on the block's
// rows, and the block's part of p_s^T q_s.
template <bool kMulti>
__global__ void __launch_bounds__(kRT) k_pcg_matvec_rows(LevelDev L, PcgDev P, int u) {
  constexpr int kNL = kMulti ? kMaxRhs : 1;
  extern __shared__ double2 sh2[];   // (16-byte aligned: pairs of columns are read as one)
  double* sh = reinterpret_cast<double*>(sh2);
  __shared__ int lc[kMaxRhs];
  __shared__ double bet[kMaxRhs];
  if (P.sc[0].all_done) return;
  const int it = P.sc[0].it_base + u;
  int s, rb;
  row_task(P.nrb, s, rb);
  if (s >= L.nsub) return;
  const int ng = L.loc_ptr[s + 1] - L.loc_ptr[s] - L.nint[s];
  const int g0 = L.goff[s];
  const int r0 = rb * kRows, rows = max(0, min(kRows, ng - r0));
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // (uniform: the columns of a wave in scalar registers)
  int nl = live_columns(P, lc);
  if (nl == 0) return;
  if constexpr (!kMulti) nl = 1;
  auto col = [&](int k) -> int {
    if constexpr (kMulti) return lc[k];
    else return 0;
  };
  const size_t slot = (size_t)s * P.nrb + rb;
  if (rows == 0) {
    if (tid < nl) P.pq_part[(size_t)col(tid) * P.ld_sub + slot] = 0.0;
    return;
  }
  const int ld = pad_ld(ng, 8);   // (columns on 128-byte boundaries: a 64-row block is four whole lines)
  const double* Sg = P.Sp + P.spoff[s] + r0;
  const int lrow = min(lane, rows - 1);
  const int cq = (ng + kNW - 1) / kNW;
  const int j0 = min(ng, wave * cq), j1 = min(ng, j0 + cq);
  for (int k = 0; k < nl; ++k) {
    const int c = col(k);
    if (it >= 2) bet[k] = P.sc[c].rzs[(it - 1) & 1] / P.sc[c].rzs[(it - 2) & 1];
  }
  if (it >= 2 && blockIdx.x == 0 && tid < nl) P.sc[col(tid)].betas[min(it - 2, kMaxHist - 1)] = bet[tid];
  constexpr int nls = kNL;
  double* pl = sh;                       // ng x kNL
  double* part = sh + (size_t)ng * nls;  // kNW x kNL x 64
  // entry a of every live column on thread a: all of its loads are issued
  // before any store (the stores of p_k could alias them)
  for (int a = tid; a < ng; a += kRT) {
    const int f = g0 + a;
    const int gi = L.gam_iid[f];
    double zv[kNL], po[kNL];
#pragma unroll
    for (int k = 0; k < kNL; ++k) {
      if (k < nl) {
        const size_t ci = (size_t)col(k) * P.ld_if + gi;
        zv[k] = P.z[ci];
        po[k] = it >= 2 ? P.p[(it - 1) & 1][ci] : 0.0;
      }
    }
    const bool own = rb == 0 && (P.shf4 ? P.shf4[f].x == f : L.sh_flat[L.sh_ptr[gi]] == f);
#pragma unroll
    for (int k = 0; k < kNL; ++k) {
      if (k < nl) {
        const double pv = (it >= 2) ? zv[k] + bet[k] * po[k] : zv[k];
        pl[(size_t)a * nls + k] = pv;
        if (own) P.p[it & 1][(size_t)col(k) * P.ld_if + gi] = pv;
      }
    }
  }
  if (kMulti && nl < kNL)
    for (int t = tid; t < ng * (kNL - nl); t += kRT) pl[(size_t)(t / (kNL - nl)) * nls + nl + t % (kNL - nl)] = 0.0;
  __syncthreads();
  double acc[kNL];
#pragma unroll
  for (int k = 0; k < kNL; ++k) acc[k] = 0.0;
  row_product<kNL>(acc, Sg, lrow, ld, j0, j1, pl);
#pragma unroll
  for (int k = 0; k < kNL; ++k)
    if (k < nl) part[(wave * kNL + k) * kRows + lane] = acc[k];
  __syncthreads();
  // column k on wave k % 4: its rows summed over the waves in wave order, the
  // product stored, the block's energy by a shuffle tree
  for (int k = wave; k < nl; k += kNW) {
    double e = 0.0;
    if (lane < rows) {
      double q = part[k * kRows + lane];
#pragma unroll
      for (int w = 1; w < kNW; ++w) q += part[(w * kNL + k) * kRows + lane];
      P.qloc[(size_t)col(k) * P.ld_flat + g0 + r0 + lane] = q;
      e = pl[(size_t)(r0 + lane) * nls + k] * q;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
    if (lane == 0) P.pq_part[(size_t)col(k) * P.ld_sub + slot] = e;
  }
}

template <int kPrec> struct RowsForm;
template <> struct RowsForm<0> { using T = double; };
template <> struct RowsForm<1> { using T = float; };

// alpha; r_k = r_{k-1} - alpha sum of the sharers' q (the owner stores r_k
// and x += alpha p) and g = delta r_k for every interface entry of the
// substructure, to P.gflat; the substructure's partial r.r.  One workgroup
// per substructure, so the gathers of the sharers' products are done once
// (not by each row block of the restriction).
template <bool kMulti>
__global__ void __launch_bounds__(kRT) k_pcg_update_rows(LevelDev L, PcgDev P, int u) {
  constexpr int kNL = kMulti ? kMaxRhs : 1;
  constexpr int kGrp = kNL < 4 ? kNL : 4;
  __shared__ int lc[kMaxRhs];
  __shared__ double red[kNW];
  __shared__ double alph[kMaxRhs];
  if (P.sc[0].all_done) return;
  const int it = P.sc[0].it_base + u;   // (an iteration: u >= 0)
  const int s = blockIdx.x;
  const int ng = L.loc_ptr[s + 1] - L.loc_ptr[s] - L.nint[s];
  const int g0 = L.goff[s];
  const int tid = threadIdx.x;
  int nl = live_columns(P, lc);
  if (nl == 0) return;
  if constexpr (!kMulti) nl = 1;
  auto col = [&](int k) -> int {
    if constexpr (kMulti) return lc[k];
    else return 0;
  };
  const double* rold = P.r[(it - 1) & 1];
  double* rnew = P.r[it & 1];
  const double* p = P.p[it & 1];
  double rr[kNL];
#pragma unroll
  for (int k = 0; k < kNL; ++k) rr[k] = 0.0;
  // alpha per live column (every thread writes the same values: no barrier)
  for (int k = 0; k < nl; ++k) alph[k] = P.sc[col(k)].rzs[(it - 1) & 1] / P.sc[col(k)].pqs;
  // entry a of every live column on thread a: its loads (the sharers'
  // products, r_{k-1}) are issued before the stores of r_k
  for (int a = tid; a < ng; a += kRT) {
    const int f = g0 + a;
    const int gi = L.gam_iid[f];
    const double d = L.delta[f];
    const int4 sf = P.shf4 ? P.shf4[f] : make_int4(-1, -1, -1, -1);
    const bool own = P.shf4 ? sf.x == f : L.sh_flat[L.sh_ptr[gi]] == f;
    // four columns at a time (the loads of a group go out together; the
    // next group's follow this group's stores)
#pragma unroll
    for (int h = 0; h < kNL; h += kGrp) {
      double q[kGrp], ro[kGrp];
#pragma unroll
      for (int e = 0; e < kGrp; ++e) {
        const int k = h + e;
        if (k < nl) {
          const double* ql = P.qloc + (size_t)col(k) * P.ld_flat;
          double v;
          if (P.shf4) {
            v = ql[sf.x];
            if (sf.y >= 0) v += ql[sf.y];
            if (sf.z >= 0) v += ql[sf.z];
            if (sf.w >= 0) v += ql[sf.w];
          } else {
            v = 0.0;
            for (int m = L.sh_ptr[gi]; m < L.sh_ptr[gi + 1]; ++m) v += ql[L.sh_flat[m]];
          }
          q[e] = v;
          ro[e] = rold[(size_t)col(k) * P.ld_if + gi];
        }
      }
#pragma unroll
      for (int e = 0; e < kGrp; ++e) {
        const int k = h + e;
        if (k < nl) {
          const double ri = ro[e] - alph[k] * q[e];
          P.gflat[(size_t)col(k) * P.ld_flat + f] = d * ri;
          if (own) {
            rnew[(size_t)col(k) * P.ld_if + gi] = ri;
            rr[k] += ri * ri;
          }
        }
      }
    }
  }
  // x += alpha p by the owners, in a pass of its own so that the loads of
  // every column go out together (after the stores of r_k, which the
  // compiler may not move them across)
  for (int a = tid; a < ng; a += kRT) {
    const int f = g0 + a;
    const int gi = L.gam_iid[f];
    if (!(P.shf4 ? P.shf4[f].x == f : L.sh_flat[L.sh_ptr[gi]] == f)) continue;
    double pv[kNL], xv[kNL];
#pragma unroll
    for (int k = 0; k < kNL; ++k) {
      if (k < nl) {
        const size_t ci = (size_t)col(k) * P.ld_if + gi;
        pv[k] = p[ci];
        xv[k] = P.x[ci];
      }
    }
#pragma unroll
    for (int k = 0; k < kNL; ++k)
      if (k < nl) P.x[(size_t)col(k) * P.ld_if + gi] = xv[k] + alph[k] * pv[k];
  }
  for (int k = 0; k < nl; ++k) {
    double v = 0.0;
#pragma unroll
    for (int m = 0; m < kNL; ++m)
      if (m == k) v = rr[m];   // (constant register index)
    v = wg_sum(v, red);
    if (tid == 0) {
      const int c = col(k);
      P.rr_part[(size_t)c * P.ld_sub + s] = v;
      if (s == 0) {
        P.sc[c].iters = it;
        P.sc[c].alphas[min(it - 1, kMaxHist - 1)] = alph[k];
      }
    }
  }
}

// g = delta r on the whole interface (iteration 0: from r_0; later: g of
// k_pcg_update_rows), then b = Psi^T g for the coarse dofs rb, rb + nrb_s,
// ... and delta T_rr g on the block's rows (zero on the corner rows).
template <int kPrec, bool kMulti>
__global__ void __launch_bounds__(kRT) k_pcg_restrict_rows(LevelDev L, PcgDev P, int u) {
  using T = typename RowsForm<kPrec>::T;
  constexpr int kNL = kMulti ? kMaxRhs : 1;
  extern __shared__ double2 sh2[];
  double* sh = reinterpret_cast<double*>(sh2);
  __shared__ int lc[kMaxRhs];
  if (P.sc[0].all_done) return;
  const int it = u < 0 ? 0 : P.sc[0].it_base + u;
  int s, rb;
  row_task(P.nrb, s, rb);
  if (s >= L.nsub) return;
  const int ng = L.loc_ptr[s + 1] - L.loc_ptr[s] - L.nint[s];
  const int nrb_s = (ng + kRows - 1) / kRows;
  if (rb >= max(1, nrb_s)) return;   // (no rows, no coarse dofs)
  const int g0 = L.goff[s];
  const int n_r = L.nr[s];
  const int ncs = L.coff[s + 1] - L.coff[s];
  const int r0 = rb * kRows;
  const int rows_r = max(0, min(kRows, n_r - r0));
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // (uniform: the columns of a wave in scalar registers)
  int nl = live_columns(P, lc);
  if (nl == 0) return;
  if constexpr (!kMulti) nl = 1;
  auto col = [&](int k) -> int {
    if constexpr (kMulti) return lc[k];
    else return 0;
  };
  const T* Tg = (kPrec == 0 ? reinterpret_cast<const T*>(P.Tp) : reinterpret_cast<const T*>(P.Tp32)) + P.tpoff[s] + r0;
  const int lrow = min(lane, max(rows_r, 1) - 1);
  const int cq = (n_r + kNW - 1) / kNW;
  const int j0 = min(n_r, wave * cq), j1 = min(n_r, j0 + cq);
  constexpr int nls = kNL;
  double* g = sh;                        // ng x kNL
  double* part = sh + (size_t)ng * nls;  // kNW x kNL x 64
  if (it == 0) {
    for (int t = tid; t < ng * nl; t += kRT) {
      const int k = t / ng, a = t - k * ng;
      g[(size_t)a * nls + k] = L.delta[g0 + a] * P.r[0][(size_t)col(k) * P.ld_if + L.gam_iid[g0 + a]];
    }
  } else {
    for (int t = tid; t < ng * nl; t += kRT) {
      const int k = t / ng, a = t - k * ng;
      g[(size_t)a * nls + k] = P.gflat[(size_t)col(k) * P.ld_flat + g0 + a];
    }
  }
  if (kMulti && nl < kNL)
    for (int t = tid; t < ng * (kNL - nl); t += kRT) g[(size_t)(t / (kNL - nl)) * nls + nl + t % (kNL - nl)] = 0.0;
  __syncthreads();
  // b = Psi^T g: one wave per coarse dof of this block, lanes over the
  // interface entries, each entry of Psi applied to every live column
  {
    const T* Pg = (kPrec == 0 ? reinterpret_cast<const T*>(L.Psi) : reinterpret_cast<const T*>(P.Psi32)) +
                  L.psioff[s];
    for (int kd = rb + wave * nrb_s; kd < ncs; kd += kNW * nrb_s) {
      double acc[kNL];
#pragma unroll
      for (int k = 0; k < kNL; ++k) acc[k] = 0.0;
      const T* Pk = Pg + (size_t)kd * ng;
      // the lane's entries of column kd of Psi, eight chunks of 64 at a time
      // (unconditional loads at clamped addresses, so they go out together)
      for (int a0 = 0; a0 < ng; a0 += 8 * 64) {
        T w[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) w[c] = Pk[min(a0 + lane + 64 * c, ng - 1)];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int a = a0 + lane + 64 * c;
          if (a < ng) {
            const double wv = static_cast<double>(w[c]);
            const double* ga = g + (size_t)a * nls;
#pragma unroll
            for (int k = 0; k < kNL; ++k)
              acc[k] += wv * ga[k];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kNL; ++k) {
        if (k >= nl) break;
        double v = acc[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (lane == 0) P.b[(size_t)col(k) * P.ld_cflat + L.coff[s] + kd] = v;
      }
    }
  }
  // delta T_rr g_r on the block's rows
  if (rows_r > 0) {
    double acc[kNL];
#pragma unroll
    for (int k = 0; k < kNL; ++k) acc[k] = 0.0;
    row_product<kNL>(acc, Tg, lrow, pad_ld(n_r, sizeof(T)), j0, j1, g);
#pragma unroll
    for (int k = 0; k < kNL; ++k)
      if (k < nl) part[(wave * kNL + k) * kRows + lane] = acc[k];
  }
  __syncthreads();
  const int rows = max(0, min(kRows, ng - r0));
  for (int t = tid; t < kRows * nl; t += kRT) {
    const int k = t / kRows, l = t - k * kRows;
    if (l >= rows) continue;
    double v = 0.0;
    if (l < rows_r) {
      v = part[k * kRows + l];
#pragma unroll
      for (int w = 1; w < kNW; ++w) v += part[(w * kNL + k) * kRows + l];
      v *= L.delta[g0 + r0 + l];
    }
    P.da[(size_t)col(k) * P.ld_flat + g0 + r0 + l] = v;
  }
}

// dynamic LDS of both launches: the gathered vector (ng x columns, even) and
// the wave partials
size_t pcg_rows_lds(int ngmax, int nrhs) {
  const size_t kNL = nrhs > 1 ? kMaxRhs : 1;
  return sizeof(double) * ((size_t)ngmax * kNL + (size_t)kNW * kNL * kRows);
}

int pcg_rows_blocks(int ngmax) { return (ngmax + kRows - 1) / kRows; }

static dim3 rows_grid(const LevelDev& L, const PcgDev& P) {
  return dim3((unsigned)(((L.nsub + 7) / 8) * 8 * P.nrb));
}

void launch_pcg_matvec_rows(hipStream_t st, const LevelDev& L, int ngmax, const PcgDev& P, int u) {
  const size_t lds = pcg_rows_lds(ngmax, P.nrhs);
  if (P.nrhs > 1)
    launch_kernel(k_pcg_matvec_rows<true>, rows_grid(L, P), dim3(kRT), lds, st, L, P, u);
  else
    launch_kernel(k_pcg_matvec_rows<false>, rows_grid(L, P), dim3(kRT), lds, st, L, P, u);
}

void launch_pcg_update_rows(hipStream_t st, const LevelDev& L, const PcgDev& P, int u) {
  if (u < 0) throw std::invalid_argument("launch_pcg_update_rows: iterations only");
  if (P.nrhs > 1)
    launch_kernel(k_pcg_update_rows<true>, dim3(L.nsub), dim3(kRT), 0, st, L, P, u);
  else
    launch_kernel(k_pcg_update_rows<false>, dim3(L.nsub), dim3(kRT), 0, st, L, P, u);
}

void launch_pcg_restrict_rows(hipStream_t st, const LevelDev& L, int ngmax, const PcgDev& P, int u) {
  const size_t lds = pcg_rows_lds(ngmax, P.nrhs);
  auto go = [&](auto kern) { launch_kernel(kern, rows_grid(L, P), dim3(kRT), lds, st, L, P, u); };
  const bool multi = P.nrhs > 1;
  if (P.prec == 0)
    multi ? go(k_pcg_restrict_rows<0, true>) : go(k_pcg_restrict_rows<0, false>);
  else
    multi ? go(k_pcg_restrict_rows<1, true>) : go(k_pcg_restrict_rows<1, false>);
}

}  // namespace bddc
