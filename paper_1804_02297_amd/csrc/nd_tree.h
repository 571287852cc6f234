// Geometric nested dissection of the n^3 grid, shared by the host and the
// GPU multifrontal factorisations of the sparsified system S.
//
// Paper: the sparse system assembled from the local rows is factored by
// nested dissection (end of Section 3.1; costs in Section 3.3).  Separators
// are planes of thickness one, which separate a 27-point stencil; the front
// of a node is its pivot points (the separator, or every point of a leaf's
// box) followed by its boundary points (the one-point shell of its box,
// which lies on ancestor separators).  Point lists are sorted global indices
// p = (i1 n + i2) n + i3; a point's three unknowns sit at front positions
// 3 a + c (a = position of the point, c = field component).
#pragma once

#include <vector>

namespace ls {

constexpr int kLeafPoints = 64;   // boxes of at most this many points are leaves

struct NdNode {
  int lo[3], hi[3];
  int child[2] = {-1, -1};
  int parent = -1;
  int depth = 0;
  std::vector<int> piv, bnd;      // sorted global point indices
  int np = 0, nb = 0;             // unknowns: 3 |piv|, 3 |bnd|
};

struct NdTree {
  int n = 0;
  int root = -1;
  int max_depth = 0;
  std::vector<NdNode> nodes;      // children are created after their parent
};

// Dissection of the whole n^3 grid.
NdTree nd_build(int n);

// position of p in the sorted list v, or -1
int nd_pos_in(const std::vector<int>& v, int p);
// front position of point p at node nd (pivots first, then boundary), or -1
int nd_front_pos(const NdNode& nd, int p);

}  // namespace ls
