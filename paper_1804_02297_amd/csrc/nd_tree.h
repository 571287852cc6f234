// Geometric nested dissection of the n^3 grid (and of the n x n grid of the
// 2-D variant, a grid of extent 1 in the third dimension), shared by the
// host and the GPU multifrontal factorisations of the sparsified system S.
//
// Paper: the sparse system assembled from the local rows is factored by
// nested dissection (end of Section 3.1; costs in Section 3.3).  Separators
// are planes of thickness one, which separate a 27-point stencil; the front
// of a node is its pivot points (the separator, or every point of a leaf's
// box) followed by its boundary points (the one-point shell of its box,
// which lies on ancestor separators).  Point lists are sorted global indices
// p = (i1 d1 + i2) d2 + i3 for grid extents (d0, d1, d2); a point's nc
// unknowns (nc = 3 field components in 3-D, 2 in 2-D) sit at front
// positions nc a + c (a = position of the point, c = field component).
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
  int np = 0, nb = 0;             // unknowns: nc |piv|, nc |bnd|
};

struct NdTree {
  int n = 0;                      // d0 (= d1 = d2 for the cube)
  int dims[3] = {0, 0, 0};
  int nc = 3;
  int root = -1;
  int max_depth = 0;
  std::vector<NdNode> nodes;      // children are created after their parent
};

// Dissection of the whole n^3 grid, three unknowns per point.
NdTree nd_build(int n);
// Dissection of a d0 x d1 x d2 grid with nc unknowns per point.
NdTree nd_build_grid(const int dims[3], int nc);

// position of p in the sorted list v, or -1
int nd_pos_in(const std::vector<int>& v, int p);
// front position of point p at node nd (pivots first, then boundary), or -1
int nd_front_pos(const NdNode& nd, int p);

}  // namespace ls
