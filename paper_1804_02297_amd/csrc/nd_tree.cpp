// Geometric nested dissection (see nd_tree.h).
#include "nd_tree.h"

#include <algorithm>

namespace ls {

namespace {

int build(NdTree& t, const int lo[3], const int hi[3], int parent, int depth) {
  const int* dm = t.dims;
  NdNode nd;
  for (int d = 0; d < 3; ++d) {
    nd.lo[d] = lo[d];
    nd.hi[d] = hi[d];
  }
  nd.parent = parent;
  nd.depth = depth;
  t.max_depth = std::max(t.max_depth, depth);
  long len[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
  const long vol = len[0] * len[1] * len[2];
  int dsplit = 0;
  for (int d = 1; d < 3; ++d)
    if (len[d] > len[dsplit]) dsplit = d;
  const bool leaf = vol <= kLeafPoints || len[dsplit] <= 2;
  const int mid = lo[dsplit] + (int)(len[dsplit] / 2);
  for (int a = lo[0]; a < hi[0]; ++a)
    for (int b = lo[1]; b < hi[1]; ++b)
      for (int c = lo[2]; c < hi[2]; ++c) {
        const int q[3] = {a, b, c};
        if (leaf || q[dsplit] == mid) nd.piv.push_back((a * dm[1] + b) * dm[2] + c);
      }
  for (int a = std::max(0, lo[0] - 1); a < std::min(dm[0], hi[0] + 1); ++a)
    for (int b = std::max(0, lo[1] - 1); b < std::min(dm[1], hi[1] + 1); ++b)
      for (int c = std::max(0, lo[2] - 1); c < std::min(dm[2], hi[2] + 1); ++c) {
        const bool inside = a >= lo[0] && a < hi[0] && b >= lo[1] && b < hi[1] && c >= lo[2] && c < hi[2];
        if (!inside) nd.bnd.push_back((a * dm[1] + b) * dm[2] + c);
      }
  nd.np = t.nc * (int)nd.piv.size();
  nd.nb = t.nc * (int)nd.bnd.size();
  const int id = (int)t.nodes.size();
  t.nodes.push_back(std::move(nd));
  if (!leaf) {
    int l_hi[3] = {hi[0], hi[1], hi[2]};
    int r_lo[3] = {lo[0], lo[1], lo[2]};
    l_hi[dsplit] = mid;
    r_lo[dsplit] = mid + 1;
    int c0 = -1, c1 = -1;
    if (mid > lo[dsplit]) c0 = build(t, lo, l_hi, id, depth + 1);
    if (mid + 1 < hi[dsplit]) c1 = build(t, r_lo, hi, id, depth + 1);
    t.nodes[id].child[0] = c0;
    t.nodes[id].child[1] = c1;
  }
  return id;
}

}  // namespace

NdTree nd_build_grid(const int dims[3], int nc) {
  NdTree t;
  t.n = dims[0];
  for (int d = 0; d < 3; ++d) t.dims[d] = dims[d];
  t.nc = nc;
  const int lo[3] = {0, 0, 0};
  t.root = build(t, lo, dims, -1, 0);
  return t;
}

NdTree nd_build(int n) {
  const int dims[3] = {n, n, n};
  return nd_build_grid(dims, 3);
}

int nd_pos_in(const std::vector<int>& v, int p) {
  auto it = std::lower_bound(v.begin(), v.end(), p);
  return (it != v.end() && *it == p) ? int(it - v.begin()) : -1;
}

int nd_front_pos(const NdNode& nd, int p) {
  int k = nd_pos_in(nd.piv, p);
  if (k >= 0) return k;
  k = nd_pos_in(nd.bnd, p);
  return k >= 0 ? (int)nd.piv.size() + k : -1;
}

}  // namespace ls
