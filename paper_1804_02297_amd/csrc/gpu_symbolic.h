// Symbolic phase of the GPU multifrontal factor (host code): the nested
// dissection, elimination order, offsets of every front's factor blocks and
// the integer index maps the device kernels use.
#pragma once

#include <cstddef>
#include <memory>
#include <new>
#include <utility>
#include <vector>

#include "../../include/ls.h"

namespace ls {

constexpr int kT = 48;                 // diagonal tile (pivot search window)
constexpr int kTileElems = kT * kT;
constexpr int kOB = 4 * kT;            // outer block: the trailing matrix is updated once per kOB pivot columns
constexpr int kSB = kOB;               // solve super-tile: four factor tiles

// One front, as the device kernels see it (offsets in elements).
struct FrontDev {
  int np, nb, nf, e0;   // pivot / boundary / front unknowns; first elimination index
  int child[2];
  long f;    // front in its level buffer: re plane [nf][nf], then the im plane
  long p;    // factor: pivot rows [np][nf] (re plane, then im plane)
  long l;    // factor: boundary rows' pivot columns [nb][np] (re, then im)
  long t;    // factor: per tile Linv re, Linv im, Uinv re, Uinv im, each [kT][kT]
  long pv;   // ints: per pivot, the tile row it was taken from
  long am;   // ints: pivot rows, 27 front point positions per pivot point (-1: none)
  long ab;   // ints: boundary rows, 27 pivot point positions per boundary point
  long bp;   // ints: boundary point list (global point indices)
  long xm;   // ints: boundary point a -> parent front point position
  long bm;   // ints: boundary unknown j -> elimination index
  long u;    // solve: first row of the node's update vector
  long m;    // factor: per super-block forward map M (z = M x on the block), [kSB][kSB] re, then im
  long h;    // factor: per super-block backward map H = U_block^-1, same layout
};

// Leaves ints uninitialised on resize: the index maps (hundreds of MB at the
// largest grids) are cleared by several threads instead of one.
template <typename T>
struct NoInitAlloc : std::allocator<T> {
  template <typename U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <typename U>
  NoInitAlloc(const NoInitAlloc<U>&) {}
  template <typename U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <typename U, typename... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};
using IntMap = std::vector<int, NoInitAlloc<int>>;

struct GpuSymbolic {
  long N = 0;                              // nc * points unknowns
  std::vector<FrontDev> fh;                // per node
  std::vector<std::vector<int>> levels;    // node ids per depth
  std::vector<long> lvl_off;               // offset of each level's list in the flattened level list
  std::vector<int> lvl_np, lvl_nf;         // largest np / nf per level
  std::vector<size_t> lvl_elems;           // level buffer elements (R) per level
  IntMap ibh;                              // every index map, [perm | per node pv, am, ab, bp, xm, bm]
  long fac_elems = 0;                      // factor elements (R)
  long u_rows = 0;                         // sum of nb over the nodes
  double flops = 0.0;                      // factorisation flops
};

// The symbolic phase for a d0 x d1 x d2 grid with nc unknowns per point,
// on up to 16 host threads.  LS_EINVAL if a map is inconsistent (checked
// after the fill), LS_ENOMEM if the maps do not fit.
ls_status gpu_symbolic(const int dims[3], int nc, GpuSymbolic& out);

}  // namespace ls
