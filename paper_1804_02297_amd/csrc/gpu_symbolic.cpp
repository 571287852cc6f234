// Symbolic phase of the GPU multifrontal factor on host threads.
//
// The dissection (nd_tree.h) fixes the fronts; this phase orders their
// pivots (deepest level first), lays out every front's factor blocks, tile
// inverses and super-block maps, and fills the integer maps the device
// kernels read: the elimination permutation, each pivot point's 27
// neighbours as front positions, each boundary point's 27 neighbours as
// pivot positions, the boundary list, its parent front positions and its
// elimination indices.  The maps of a front depend only on that front, so
// up to 16 threads take fronts from a shared counter.
#include "gpu_symbolic.h"

#include <algorithm>
#include <atomic>
#include <functional>
#include <limits>
#include <system_error>
#include <thread>

#include "nd_tree.h"

namespace ls {

namespace {

// fn() on the calling thread and up to nthr - 1 more; fn takes its work from a
// shared counter, so fewer threads (when one cannot be started) still finish it
template <typename F>
void run_on_threads(int nthr, F& fn) {
  std::vector<std::thread> workers;
  for (int i = 1; i < nthr; ++i) {
    try {
      workers.emplace_back(std::ref(fn));
    } catch (const std::system_error&) {
      break;
    }
  }
  fn();
  for (auto& th : workers) th.join();
}

// Symbolic phase: dissection, elimination order, offsets and index maps.
ls_status symbolic_impl(const int* dm, int nc, GpuSymbolic& g) {
  IntMap& ibh = g.ibh;
  long& fac_elems = g.fac_elems;
  NdTree t = nd_build_grid(dm, nc);
  const int nn = (int)t.nodes.size();
  const long n3 = (long)dm[0] * dm[1] * dm[2];
  g.N = (long)nc * n3;
  g.levels.assign(t.max_depth + 1, {});
  for (int i = 0; i < nn; ++i) g.levels[t.nodes[i].depth].push_back(i);
  g.fh.assign(nn, FrontDev{});
  // elimination order: deepest level first
  std::vector<long> elim_of_point(n3, -1);
  long e = 0;
  for (int dep = t.max_depth; dep >= 0; --dep)
    for (int id : g.levels[dep]) {
      const NdNode& nd = t.nodes[id];
      FrontDev& f = g.fh[id];
      f.np = nd.np;
      f.nb = nd.nb;
      f.nf = nd.np + nd.nb;
      f.e0 = (int)e;
      f.child[0] = nd.child[0];
      f.child[1] = nd.child[1];
      for (size_t a = 0; a < nd.piv.size(); ++a) elim_of_point[nd.piv[a]] = e + (long)nc * a;
      e += nd.np;
    }
  if (e != g.N) return LS_EINVAL;
  // int maps: perm [N], then per node pv, am, ab, bp, xm, bm
  long io = g.N;
  for (int id = 0; id < nn; ++id) {
    const NdNode& nd = t.nodes[id];
    FrontDev& f = g.fh[id];
    f.pv = io;
    io += nd.np;
    f.am = io;
    io += 27L * (long)nd.piv.size();
    f.ab = io;
    io += 27L * (long)nd.bnd.size();
    f.bp = io;
    io += (long)nd.bnd.size();
    f.xm = io;
    io += (long)nd.bnd.size();
    f.bm = io;
    io += nd.nb;
  }
  if (io > (long)std::numeric_limits<int>::max()) return LS_ENOMEM;
  const int nthr = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  try {
    ibh.resize(io);
  } catch (const std::bad_alloc&) {
    return LS_ENOMEM;
  }
  std::atomic<long> next_chunk{0};
  constexpr long kChunk = 1L << 20;
  auto clear_maps = [&]() {
    for (long c = next_chunk.fetch_add(1); c * kChunk < io; c = next_chunk.fetch_add(1))
      std::fill(ibh.begin() + c * kChunk, ibh.begin() + std::min(io, (c + 1) * kChunk), -1);
  };
  run_on_threads(nthr, clear_maps);
  // The maps of a front depend only on that front, so fronts are taken from a
  // shared counter by host threads; each front writes its own ranges of ibh.
  // A thread keeps a point -> front-position table (pivots first, then the
  // boundary; -1 elsewhere), set for the current front and cleared after it,
  // so the 27 neighbour lookups per point are direct loads.
  std::atomic<int> next_front{0};
  std::atomic<bool> bad{false};
  auto fill_fronts = [&]() {
    std::vector<int> pos;
    try {
      pos.assign(n3, -1);
    } catch (const std::bad_alloc&) {
      return;   // the other threads take the fronts; none left untaken is checked below
    }
    for (int id = next_front.fetch_add(1); id < nn && !bad.load(std::memory_order_relaxed);
         id = next_front.fetch_add(1)) {
      const NdNode& nd = t.nodes[id];
      const FrontDev& f = g.fh[id];
      const int npp = (int)nd.piv.size();
      for (size_t b = 0; b < nd.bnd.size(); ++b) pos[nd.bnd[b]] = npp + (int)b;
      for (int a = 0; a < npp; ++a) pos[nd.piv[a]] = a;   // a pivot position wins, as in nd_front_pos
      for (int a = 0; a < npp; ++a)
        for (int c = 0; c < nc; ++c) ibh[f.e0 + nc * a + c] = (int)(c * n3 + nd.piv[a]);
      // neighbours of point p: their front positions (pivot rows) or pivot positions (boundary rows)
      auto nb_map = [&](int p, long dst, bool pivot_row) {
        const int i3 = p % dm[2], i2 = (p / dm[2]) % dm[1], i1 = p / (dm[1] * dm[2]);
        for (int s1 = -1; s1 <= 1; ++s1)
          for (int s2 = -1; s2 <= 1; ++s2)
            for (int s3 = -1; s3 <= 1; ++s3) {
              const int slot = 9 * (s1 + 1) + 3 * (s2 + 1) + (s3 + 1);
              const int j1 = i1 + s1, j2 = i2 + s2, j3 = i3 + s3;
              int v = -1;
              if (j1 >= 0 && j1 < dm[0] && j2 >= 0 && j2 < dm[1] && j3 >= 0 && j3 < dm[2]) {
                const int q = pos[(j1 * dm[1] + j2) * dm[2] + j3];
                v = (pivot_row || q < npp) ? q : -1;
              }
              ibh[dst + slot] = v;
            }
      };
      for (int a = 0; a < npp; ++a) nb_map(nd.piv[a], f.am + 27L * a, true);
      for (size_t b = 0; b < nd.bnd.size(); ++b) {
        nb_map(nd.bnd[b], f.ab + 27L * b, false);
        ibh[f.bp + b] = nd.bnd[b];
        const long eb = elim_of_point[nd.bnd[b]];
        if (eb < 0) bad = true;
        for (int c = 0; c < nc; ++c) ibh[f.bm + nc * b + c] = (int)(eb + c);
      }
      if (nd.parent >= 0) {
        const NdNode& pa = t.nodes[nd.parent];
        for (size_t b = 0; b < nd.bnd.size(); ++b) {
          const int fp = nd_front_pos(pa, nd.bnd[b]);
          if (fp < 0) bad = true;               // a child's shell lies in its parent's front
          ibh[f.xm + b] = fp;
        }
      }
      for (int a = 0; a < npp; ++a) pos[nd.piv[a]] = -1;
      for (size_t b = 0; b < nd.bnd.size(); ++b) pos[nd.bnd[b]] = -1;
    }
  };
  run_on_threads(nthr, fill_fronts);
  if (bad) return LS_EINVAL;
  if (next_front.load() < nn) return LS_ENOMEM;   // no thread could allocate its table
  // factor offsets (R elements) and solve update rows
  long fo = 0, uo = 0;
  double fl = 0.0;
  for (int id = 0; id < nn; ++id) {
    FrontDev& f = g.fh[id];
    const long np = f.np, nb = f.nb, nf = f.nf;
    f.p = fo;
    fo += 2 * np * nf;
    f.l = fo;
    fo += 2 * nb * np;
    f.t = fo;
    fo += 4L * kTileElems * ((np + kT - 1) / kT);
    f.m = fo;
    fo += 2L * kSB * kSB * ((np + kSB - 1) / kSB);
    f.h = fo;
    fo += 2L * kSB * kSB * ((np + kSB - 1) / kSB);
    f.u = uo;
    uo += nb;
    for (long kb = 0; kb < np; kb += kT) {
      const long ke = std::min(np, kb + kT), rows = nf - ke;
      fl += 8.0 * (double)rows * (double)rows * (double)(ke - kb);
    }
  }
  fac_elems = fo;
  g.u_rows = uo;
  g.flops = fl;
  // level buffers and per-level extents
  const int L = (int)g.levels.size();
  g.lvl_off.assign(L, 0);
  g.lvl_np.assign(L, 0);
  g.lvl_nf.assign(L, 0);
  g.lvl_elems.assign(L, 0);
  long lo = 0;
  for (int dep = 0; dep < L; ++dep) {
    g.lvl_off[dep] = lo;
    lo += (long)g.levels[dep].size();
    size_t off = 0;
    for (int id : g.levels[dep]) {
      FrontDev& f = g.fh[id];
      f.f = (long)off;
      off += 2 * (size_t)f.nf * f.nf;
      g.lvl_np[dep] = std::max(g.lvl_np[dep], f.np);
      g.lvl_nf[dep] = std::max(g.lvl_nf[dep], f.nf);
    }
    g.lvl_elems[dep] = off;
  }
  // every map entry in range (checked once here, after the fill; the kernels trust them)
  next_front = 0;
  auto check_fronts = [&]() {
    for (int id = next_front.fetch_add(1); id < nn; id = next_front.fetch_add(1)) {
      const FrontDev& f = g.fh[id];
      const NdNode& nd = t.nodes[id];
      bool ok = true;
      for (long i = 0; i < 27L * (long)nd.piv.size(); ++i) ok &= ibh[f.am + i] < f.nf / nc;
      for (long i = 0; i < 27L * (long)nd.bnd.size(); ++i) ok &= ibh[f.ab + i] < f.np / nc;
      if (nd.parent >= 0)
        for (size_t b = 0; b < nd.bnd.size(); ++b) ok &= ibh[f.xm + b] < g.fh[nd.parent].nf / nc;
      if (!ok) bad = true;
    }
  };
  run_on_threads(nthr, check_fronts);
  if (bad) return LS_EINVAL;
  return LS_OK;
}


}  // namespace

ls_status gpu_symbolic(const int dims[3], int nc, GpuSymbolic& out) {
  if (!dims || dims[0] < 1 || dims[1] < 1 || dims[2] < 1 || (nc != 2 && nc != 3)) return LS_EINVAL;
  try {
    return symbolic_impl(dims, nc, out);
  } catch (const std::bad_alloc&) {
    return LS_ENOMEM;
  } catch (const std::length_error&) {
    return LS_ENOMEM;
  }
}

}  // namespace ls
