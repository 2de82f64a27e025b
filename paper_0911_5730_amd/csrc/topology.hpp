// Host-side substructure topology of one decomposition level (integer work).
//
// Section 2: substructures share interface dofs; coarse dofs are corner values
// and edge functionals.  Section 2.1: at level l the elements are the level-(l-1)
// substructures and the dofs are the level-(l-1) coarse dofs, so the same
// classification runs at every level on an element -> dof incidence.
//
// Classification (the paper assumes a conforming triangulation and asks only for
// "sufficient" corners, Section 5):
//   interface dof: shared by >= 2 substructures; corner: shared by >= 3;
//   edge of the pair (s,t): every non-corner dof shared by exactly s and t;
//   a pair with a floating member that shares no corner gets the lowest dof
//   of its edge promoted to a corner; a floating substructure with no corner
//   gets the lowest dof of its largest edge promoted.
#pragma once

#include <array>
#include <cstdint>
#include <memory>
#include <vector>

namespace bddc {

constexpr int kMaxShare = 4;   // substructures that may share one dof (a node of a 2D quad mesh touches <= 4 elements)

struct Topology {
  int n = 0;                        // dofs of the level
  int nsub = 0;
  std::vector<uint8_t> nshare;      // |N_d|
  std::unique_ptr<int32_t[]> share_;  // N_d, ascending: share(d)[0 .. nshare[d])
  const int32_t* share(int d) const { return share_.get() + (size_t)d * kMaxShare; }
  std::vector<uint8_t> is_corner;
  std::vector<uint8_t> floating;    // per substructure: no Dirichlet contact
  // local dofs of each substructure ordered [interior | interface non-corner | corner]; inside each
  // group the order is that of first appearance in the substructure's elements (ascending element id)
  std::vector<int32_t> loc_ptr, loc_dof;
  std::vector<int32_t> n_int, n_r, n_c;
  std::vector<int32_t> corners;     // ascending
  std::vector<int32_t> edge_s, edge_t, edge_ptr, edge_dof;   // edges in (s,t) order, dofs ascending
  int n_interface = 0;

  int nedges() const { return static_cast<int>(edge_s.size()); }
  int nloc(int s) const { return loc_ptr[s + 1] - loc_ptr[s]; }
  int ngam(int s) const { return n_r[s] + n_c[s]; }
};

// elements given as CSR (elem_ptr, elem_dof); elem_sub[e] in [0, nsub);
// elem_touch[e] != 0 if the element carries Dirichlet data (its substructure does not float).
// Throws Error{BDDC_EPARTITION} on an empty substructure, too many sharers,
// or (require_connected) a substructure whose elements with dofs do not form
// one piece connected through shared dofs.
Topology classify(int n, int nsub, const std::vector<int32_t>& elem_ptr,
                  const std::vector<int32_t>& elem_dof, const std::vector<int32_t>& elem_sub,
                  const std::vector<uint8_t>& elem_touch, bool require_connected = false);

// The rules above applied to given sharer lists (T.nshare, T.share_), floating
// flags and each substructure's dof list (raw_ptr, raw): corners, edges and the
// local ordering.
void classify_rules(Topology& T, const std::vector<int32_t>& raw_ptr, const std::vector<int32_t>& raw);

// Assembly maps of the level-1 grid: elements of each substructure in
// ascending id (sub_el_ptr, el_gid), the local position of each element node
// (el_loc, 4 per element, -1 for Dirichlet nodes) and for each local dof the
// (local element << 2 | corner) entries of its elements (node_el, 4 per dof,
// -1 padded, elements in ascending id).
struct GridMaps {
  std::vector<int32_t> sub_el_ptr, el_gid, el_loc, node_el;
  int per_el = 4;      // entries of el_loc per element (element dofs)
  int pos_bits = 2;    // node_el entries: (local element << pos_bits) | position in the element
};

// Level 1 on the nx x ny element grid of the unit square with zero Dirichlet
// data on the boundary: free node (i, j), 1 <= i < nx, 1 <= j < ny, has id
// (j-1)(nx-1) + (i-1); element (i, j) has id j nx + i and nodes (i,j), (i+1,j),
// (i+1,j+1), (i,j+1).  The sharers of a node are the parts of its four
// elements, so everything is computed node by node; each substructure's dofs
// are taken in ascending id.  Same rules and errors as classify; maps may be null.
Topology classify_grid(int nx, int ny, const int32_t* part, int nsub, GridMaps* maps);

// Vector problems with dpn dofs per node (plane elasticity: dpn = 2): the
// node topology of classify_grid turned into the dof topology in place --
// node d becomes dofs dpn d .. dpn d + dpn - 1 with its sharers, its class
// (interior, edge, corner) and its place in each local ordering; the maps
// list the element dofs node by node (position dpn q + c for component c of
// the element's node q).
void expand_node_topology(Topology& T, GridMaps* maps, int dpn);

}  // namespace bddc
