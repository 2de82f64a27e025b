// Host-side substructure topology (see topology.hpp for the classification rules).
#include "topology.hpp"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <unordered_set>

#include "common.hpp"

namespace bddc {

namespace {
inline uint64_t pair_key(int s, int t) {
  return (static_cast<uint64_t>(static_cast<uint32_t>(s)) << 32) | static_cast<uint32_t>(t);
}
}  // namespace

Topology classify(int n, int nsub, const std::vector<int32_t>& elem_ptr,
                  const std::vector<int32_t>& elem_dof, const std::vector<int32_t>& elem_sub,
                  const std::vector<uint8_t>& elem_touch, bool require_connected) {
  const bool timing = getenv("BDDC_HOST_TIMING") != nullptr;
  auto t0 = std::chrono::steady_clock::now();
  auto lap = [&](const char* what) {
    if (!timing) return;
    const auto now = std::chrono::steady_clock::now();
    fprintf(stderr, "libbddc classify %-12s %8.3f ms\n", what, std::chrono::duration<double, std::milli>(now - t0).count());
    t0 = now;
  };
  Topology T;
  T.n = n;
  T.nsub = nsub;
  T.nshare.assign(n, 0);
  T.share_.reset(new int32_t[(size_t)std::max(n, 1) * kMaxShare]);
  int32_t* share = T.share_.get();
  T.floating.assign(nsub, 1);
  T.is_corner.assign(n, 0);
  const int ne = static_cast<int>(elem_sub.size());

  // elements grouped by substructure (stable counting sort)
  std::vector<int32_t> sptr(nsub + 1, 0), order(ne);
  for (int e = 0; e < ne; ++e) sptr[elem_sub[e] + 1]++;
  for (int s = 0; s < nsub; ++s) {
    if (sptr[s + 1] == 0) fail(BDDC_EPARTITION, "substructure " + std::to_string(s) + " owns no element");
    sptr[s + 1] += sptr[s];
  }
  {
    std::vector<int32_t> pos(sptr.begin(), sptr.end() - 1);
    for (int e = 0; e < ne; ++e) order[pos[elem_sub[e]]++] = e;
  }
  lap("group");

  // N_d (ascending because substructures are visited in order) and raw local dof lists
  std::vector<int32_t> mark(n, -1);
  std::vector<int32_t> raw_ptr(nsub + 1, 0), raw;
  raw.reserve(elem_dof.size());
  for (int s = 0; s < nsub; ++s) {
    for (int k = sptr[s]; k < sptr[s + 1]; ++k) {
      const int e = order[k];
      if (elem_touch[e]) T.floating[s] = 0;
      for (int q = elem_ptr[e]; q < elem_ptr[e + 1]; ++q) {
        const int d = elem_dof[q];
        if (mark[d] == s) continue;
        mark[d] = s;
        if (T.nshare[d] >= kMaxShare) fail(BDDC_EUNSUPPORTED, "a dof is shared by too many substructures");
        share[(size_t)d * kMaxShare + T.nshare[d]++] = s;
        raw.push_back(d);
      }
    }
    raw_ptr[s + 1] = static_cast<int32_t>(raw.size());
  }
  lap("sharers");
  if (require_connected) {
    // every substructure connected through its dofs (elements without dofs
    // left out): a disconnected one would have a null space per piece, which
    // the corners of the rules below do not remove
    std::vector<int32_t> up(ne), first(n, -1);
    for (int e = 0; e < ne; ++e) up[e] = e;
    auto root = [&](int x) {
      while (up[x] != x) x = up[x] = up[up[x]];
      return x;
    };
    for (int s = 0; s < nsub; ++s) {
      for (int k = sptr[s]; k < sptr[s + 1]; ++k) {
        const int e = order[k];
        for (int q = elem_ptr[e]; q < elem_ptr[e + 1]; ++q) {
          const int d = elem_dof[q];
          if (first[d] < 0 || elem_sub[first[d]] != s) {
            first[d] = e;
          } else {
            const int a = root(e), b = root(first[d]);
            if (a != b) up[a] = b;
          }
        }
      }
      int pieces = 0, r0 = -1;
      for (int k = sptr[s]; k < sptr[s + 1]; ++k) {
        const int e = order[k];
        if (elem_ptr[e + 1] == elem_ptr[e]) continue;
        const int r = root(e);
        if (r0 < 0) r0 = r, pieces = 1;
        else if (r != r0) pieces = 2;
      }
      if (pieces > 1)
        fail(BDDC_EPARTITION, "substructure " + std::to_string(s) + " of a coarse level is not connected through its dofs");
    }
    lap("connected");
  }
  classify_rules(T, raw_ptr, raw);
  lap("rules");
  return T;
}

void classify_rules(Topology& T, const std::vector<int32_t>& raw_ptr, const std::vector<int32_t>& raw) {
  const int n = T.n, nsub = T.nsub;
  // corners and edge candidates, ordered by (s, t, dof): counting sort by s
  // (dofs visited in increasing order), then a small sort by t inside each bucket
  std::vector<int32_t> bcnt(nsub + 1, 0);
  size_t ncand = 0;
  for (int d = 0; d < n; ++d) {
    if (T.nshare[d] >= 3) T.is_corner[d] = 1;
    else if (T.nshare[d] == 2) { bcnt[T.share(d)[0] + 1]++; ++ncand; }
  }
  for (int s = 0; s < nsub; ++s) bcnt[s + 1] += bcnt[s];
  std::vector<std::pair<uint64_t, int32_t>> cand(ncand);
  {
    std::vector<int32_t> pos(bcnt.begin(), bcnt.end() - 1);
    for (int d = 0; d < n; ++d)
      if (T.nshare[d] == 2) cand[pos[T.share(d)[0]]++] = {pair_key(T.share(d)[0], T.share(d)[1]), d};
  }
  for (int s = 0; s < nsub; ++s)
    std::stable_sort(cand.begin() + bcnt[s], cand.begin() + bcnt[s + 1],
                     [](const std::pair<uint64_t, int32_t>& a, const std::pair<uint64_t, int32_t>& b) {
                       return a.first < b.first;
                     });
  // groups of candidates by pair
  std::vector<size_t> gstart;
  for (size_t i = 0; i < cand.size(); ++i)
    if (i == 0 || cand[i].first != cand[i - 1].first) gstart.push_back(i);
  gstart.push_back(cand.size());
  const size_t ng = gstart.size() - 1;
  std::vector<uint8_t> removed(cand.size(), 0);

  std::unordered_set<uint64_t> covered;
  for (int d = 0; d < n; ++d) {
    if (!T.is_corner[d]) continue;
    for (int a = 0; a < T.nshare[d]; ++a)
      for (int b = a + 1; b < T.nshare[d]; ++b) covered.insert(pair_key(T.share(d)[a], T.share(d)[b]));
  }
  // rule: a pair with a floating member shares at least one corner
  for (size_t g = 0; g < ng; ++g) {
    const uint64_t key = cand[gstart[g]].first;
    const int s = static_cast<int>(key >> 32), t = static_cast<int>(key & 0xffffffffu);
    if (!(T.floating[s] || T.floating[t])) continue;
    if (covered.count(key)) continue;
    const size_t i = gstart[g];   // lowest dof of the group
    T.is_corner[cand[i].second] = 1;
    removed[i] = 1;
    covered.insert(key);
  }
  // rule: a floating substructure owns at least one corner
  for (int s = 0; s < nsub; ++s) {
    if (!T.floating[s]) continue;
    bool has = false;
    for (int k = raw_ptr[s]; k < raw_ptr[s + 1] && !has; ++k) has = T.is_corner[raw[k]] != 0;
    if (has) continue;
    long best = -1;
    size_t bestg = 0;
    for (size_t g = 0; g < ng; ++g) {
      const uint64_t key = cand[gstart[g]].first;
      const int a = static_cast<int>(key >> 32), b = static_cast<int>(key & 0xffffffffu);
      if (a != s && b != s) continue;
      long cnt = 0;
      for (size_t i = gstart[g]; i < gstart[g + 1]; ++i) cnt += !removed[i];
      if (cnt > best) { best = cnt; bestg = g; }
    }
    if (best <= 0) fail(BDDC_EPARTITION, "floating substructure " + std::to_string(s) + " has no interface");
    for (size_t i = gstart[bestg]; i < gstart[bestg + 1]; ++i)
      if (!removed[i]) { T.is_corner[cand[i].second] = 1; removed[i] = 1; break; }
  }

  // final edges
  T.edge_ptr.push_back(0);
  for (size_t g = 0; g < ng; ++g) {
    size_t before = T.edge_dof.size();
    for (size_t i = gstart[g]; i < gstart[g + 1]; ++i)
      if (!removed[i]) T.edge_dof.push_back(cand[i].second);
    if (T.edge_dof.size() == before) continue;
    const uint64_t key = cand[gstart[g]].first;
    T.edge_s.push_back(static_cast<int32_t>(key >> 32));
    T.edge_t.push_back(static_cast<int32_t>(key & 0xffffffffu));
    T.edge_ptr.push_back(static_cast<int32_t>(T.edge_dof.size()));
  }
  for (int d = 0; d < n; ++d) {
    if (T.is_corner[d]) T.corners.push_back(d);
    if (T.nshare[d] >= 2) T.n_interface++;
  }

  // local ordering [interior | interface non-corner | corner], each group in the order of raw
  T.loc_ptr.assign(nsub + 1, 0);
  T.n_int.assign(nsub, 0);
  T.n_r.assign(nsub, 0);
  T.n_c.assign(nsub, 0);
  T.loc_dof.resize(raw.size());
  parallel_for(nsub, 8, [&](int s0, int s1) {
  for (int s = s0; s < s1; ++s) {
    int ni = 0, nr = 0, nc = 0;
    for (int k = raw_ptr[s]; k < raw_ptr[s + 1]; ++k) {
      const int d = raw[k];
      if (T.nshare[d] == 1) ++ni;
      else if (T.is_corner[d]) ++nc;
      else ++nr;
    }
    T.n_int[s] = ni;
    T.n_r[s] = nr;
    T.n_c[s] = nc;
    const int b = raw_ptr[s];
    T.loc_ptr[s] = b;
    int oi = b, orr = b + ni, oc = b + ni + nr;
    for (int k = raw_ptr[s]; k < raw_ptr[s + 1]; ++k) {
      const int d = raw[k];
      if (T.nshare[d] == 1) T.loc_dof[oi++] = d;
      else if (T.is_corner[d]) T.loc_dof[oc++] = d;
      else T.loc_dof[orr++] = d;
    }
  }
  });
  T.loc_ptr[nsub] = raw_ptr[nsub];
}

Topology classify_grid(int nx, int ny, const int32_t* part, int nsub, GridMaps* maps) {
  const bool timing = getenv("BDDC_HOST_TIMING") != nullptr;
  auto t0 = std::chrono::steady_clock::now();
  auto lap = [&](const char* what) {
    if (!timing) return;
    const auto now = std::chrono::steady_clock::now();
    fprintf(stderr, "libbddc classify_grid %-12s %8.3f ms\n", what, std::chrono::duration<double, std::milli>(now - t0).count());
    t0 = now;
  };
  Topology T;
  const int ne = nx * ny;
  const int mx = nx - 1;
  const int n = (nx - 1) * (ny - 1);
  T.n = n;
  T.nsub = nsub;
  T.nshare.assign(n, 0);
  T.share_.reset(new int32_t[(size_t)std::max(n, 1) * kMaxShare]);
  int32_t* share = T.share_.get();
  T.floating.assign(nsub, 1);
  T.is_corner.assign(n, 0);
  // elements per substructure; an element on the outer ring carries Dirichlet nodes
  std::vector<int32_t> ecnt(nsub + 1, 0);
  for (int e = 0; e < ne; ++e) {
    const int s = part[e];
    if (s < 0 || s >= nsub) fail(BDDC_EPARTITION, "part entries must lie in [0, nsub)");
    ecnt[s + 1]++;
  }
  for (int s = 0; s < nsub; ++s) {
    if (ecnt[s + 1] == 0) fail(BDDC_EPARTITION, "substructure " + std::to_string(s) + " owns no element");
    ecnt[s + 1] += ecnt[s];
  }
  for (int i = 0; i < nx; ++i) {
    T.floating[part[i]] = 0;
    T.floating[part[(ny - 1) * nx + i]] = 0;
  }
  for (int j = 0; j < ny; ++j) {
    T.floating[part[j * nx]] = 0;
    T.floating[part[j * nx + nx - 1]] = 0;
  }
  lap("elements");
  // N_d from the four elements around node (i, j): (i-1,j-1), (i,j-1), (i-1,j), (i,j)
  parallel_for(ny - 1, 8, [&](int r0, int r1) {
    for (int j = r0 + 1; j <= r1; ++j)
      for (int i = 1; i < nx; ++i) {
        const int d = (j - 1) * mx + (i - 1);
        const int p4[4] = {part[(j - 1) * nx + i - 1], part[(j - 1) * nx + i], part[j * nx + i - 1], part[j * nx + i]};
        int32_t* sh = share + (size_t)d * kMaxShare;
        int m = 0;
        for (int q = 0; q < 4; ++q) {
          int k = 0;
          while (k < m && sh[k] < p4[q]) ++k;
          if (k < m && sh[k] == p4[q]) continue;
          for (int r = m; r > k; --r) sh[r] = sh[r - 1];
          sh[k] = p4[q];
          ++m;
        }
        T.nshare[d] = (uint8_t)m;
      }
  });
  std::vector<int32_t> rcnt(nsub + 1, 0);
  for (int d = 0; d < n; ++d)
    for (int k = 0; k < T.nshare[d]; ++k) rcnt[T.share(d)[k] + 1]++;
  // each substructure's dofs in ascending order
  for (int s = 0; s < nsub; ++s) rcnt[s + 1] += rcnt[s];
  std::vector<int32_t> raw_ptr(rcnt), raw(rcnt[nsub]);
  {
    std::vector<int32_t> pos(rcnt.begin(), rcnt.end() - 1);
    for (int d = 0; d < n; ++d)
      for (int k = 0; k < T.nshare[d]; ++k) raw[pos[T.share(d)[k]]++] = d;
  }
  lap("sharers");
  classify_rules(T, raw_ptr, raw);
  lap("rules");
  if (!maps) return T;
  // assembly maps: elements per substructure (ascending), the local position of
  // each element node, and for each local dof the (element, corner) pairs
  GridMaps& M = *maps;
  M.sub_el_ptr = ecnt;
  M.el_gid.resize(ne);
  std::vector<int32_t> loc_e(ne);
  {
    std::vector<int32_t> pos(ecnt.begin(), ecnt.end() - 1);
    for (int e = 0; e < ne; ++e) {
      const int s = part[e];
      loc_e[e] = pos[s] - ecnt[s];
      M.el_gid[pos[s]++] = e;
    }
  }
  lap("el_gid");
  // posk[d * kMaxShare + k]: local position of d in its k-th sharer
  std::vector<int32_t> posk((size_t)n * kMaxShare, -1);
  parallel_for(nsub, 4, [&](int s0, int s1) {
    for (int s = s0; s < s1; ++s) {
      const int b = T.loc_ptr[s];
      for (int a = 0; a < T.nloc(s); ++a) {
        const int d = T.loc_dof[b + a];
        const int32_t* sh = T.share(d);
        int k = 0;
        while (sh[k] != s) ++k;
        posk[(size_t)d * kMaxShare + k] = a;
      }
    }
  });
  auto pos_in = [&](int d, int s) {
    const int32_t* sh = T.share(d);
    int k = 0;
    while (sh[k] != s) ++k;
    return posk[(size_t)d * kMaxShare + k];
  };
  auto fid = [&](int i, int j) -> int {
    if (i <= 0 || j <= 0 || i >= nx || j >= ny) return -1;
    return (j - 1) * mx + (i - 1);
  };
  lap("posk");
  M.el_loc.assign((size_t)ne * 4, -1);
  M.node_el.assign((size_t)T.loc_ptr[nsub] * 4, -1);
  parallel_for(nsub, 4, [&](int s0, int s1) {
    for (int s = s0; s < s1; ++s) {
      // element nodes in local numbering
      for (int le = 0; le < ecnt[s + 1] - ecnt[s]; ++le) {
        const int e = M.el_gid[ecnt[s] + le];
        const int i = e % nx, j = e / nx;
        const int nd[4] = {fid(i, j), fid(i + 1, j), fid(i + 1, j + 1), fid(i, j + 1)};
        int32_t* el = &M.el_loc[(size_t)(ecnt[s] + le) * 4];
        for (int q = 0; q < 4; ++q) el[q] = nd[q] >= 0 ? pos_in(nd[q], s) : -1;
      }
      // for each local dof, its elements in s in ascending id with the dof's corner
      const int b = T.loc_ptr[s];
      for (int a = 0; a < T.nloc(s); ++a) {
        const int d = T.loc_dof[b + a];
        const int i = d % mx + 1, j = d / mx + 1;
        const int es[4] = {(j - 1) * nx + i - 1, (j - 1) * nx + i, j * nx + i - 1, j * nx + i};
        const int qs[4] = {2, 3, 1, 0};
        int32_t* slot = &M.node_el[(size_t)(b + a) * 4];
        int t = 0;
        for (int k = 0; k < 4; ++k)
          if (part[es[k]] == s) slot[t++] = (loc_e[es[k]] << 2) | qs[k];
      }
    }
  });
  lap("node_el");
  return T;
}

void expand_node_topology(Topology& T, GridMaps* maps, int dpn) {
  if (dpn == 1) return;
  const int nn = T.n;
  Topology D;
  D.n = dpn * nn;
  D.nsub = T.nsub;
  D.nshare.resize(D.n);
  D.share_.reset(new int32_t[(size_t)std::max(D.n, 1) * kMaxShare]);
  D.is_corner.resize(D.n);
  for (int d = 0; d < nn; ++d)
    for (int c = 0; c < dpn; ++c) {
      const int e = dpn * d + c;
      D.nshare[e] = T.nshare[d];
      for (int k = 0; k < kMaxShare; ++k) D.share_[(size_t)e * kMaxShare + k] = T.share(d)[k];
      D.is_corner[e] = T.is_corner[d];
    }
  D.floating = T.floating;
  auto scale = [&](const std::vector<int32_t>& v) {
    std::vector<int32_t> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = dpn * v[i];
    return o;
  };
  auto spread = [&](const std::vector<int32_t>& v) {   // node list -> dof list, components in order
    std::vector<int32_t> o;
    o.reserve(v.size() * dpn);
    for (int32_t d : v)
      for (int c = 0; c < dpn; ++c) o.push_back(dpn * d + c);
    return o;
  };
  D.loc_ptr = scale(T.loc_ptr);
  D.loc_dof = spread(T.loc_dof);
  D.n_int = scale(T.n_int);
  D.n_r = scale(T.n_r);
  D.n_c = scale(T.n_c);
  D.corners = spread(T.corners);
  D.edge_s = T.edge_s;
  D.edge_t = T.edge_t;
  D.edge_ptr = scale(T.edge_ptr);
  D.edge_dof = spread(T.edge_dof);
  D.n_interface = dpn * T.n_interface;
  T = std::move(D);
  if (!maps) return;
  GridMaps& M = *maps;
  const int q0 = M.per_el;
  const size_t ne = M.el_gid.size();
  std::vector<int32_t> el_loc(ne * q0 * dpn, -1);
  for (size_t e = 0; e < ne; ++e)
    for (int q = 0; q < q0; ++q) {
      const int a = M.el_loc[e * q0 + q];
      for (int c = 0; c < dpn; ++c) el_loc[(e * q0 + q) * dpn + c] = a >= 0 ? dpn * a + c : -1;
    }
  int bits = 0;
  while ((1 << bits) < q0 * dpn) ++bits;
  const size_t nloc = M.node_el.size() / 4;
  std::vector<int32_t> node_el(nloc * dpn * 4, -1);
  for (size_t a = 0; a < nloc; ++a)
    for (int c = 0; c < dpn; ++c)
      for (int k = 0; k < 4; ++k) {
        const int code = M.node_el[a * 4 + k];
        if (code < 0) continue;
        const int le = code >> M.pos_bits, q = code & ((1 << M.pos_bits) - 1);
        node_el[((a * dpn + c) * 4) + k] = (le << bits) | (q * dpn + c);
      }
  M.el_loc.swap(el_loc);
  M.node_el.swap(node_el);
  M.per_el = q0 * dpn;
  M.pos_bits = bits;
}

}  // namespace bddc
