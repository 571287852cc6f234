// Autotuner of the batched apply: for one (n, precision, batch) it times every
// launch choice on the plan's own operator and keeps the fastest.
//
// Choices:
//   * the right-hand sides per launch set (chunk: 1, 2, 4, ... up to the
//     batch): a smaller chunk trades launch count for a working set that can
//     stay in the last-level cache between passes;
//   * the pass-3 teams per workgroup (1, 2, 4 where a team is one wavefront):
//     workgroup size against phase overlap on a CU;
//   * the row-run length of each strided pass (256 or 128 bytes, the FFT tile
//     of the pass): a half tile halves the workgroup's LDS and fits more
//     workgroups per CU to cover its latency;
//   * persistent launches, for the strided passes and for pass 3 apart: a
//     pass launches only the workgroups the device holds at once, which
//     stride over the work items (pass 3 reloads its symbol line per work
//     item, and a workgroup that waits for it idles its CU unless other
//     workgroups are resident there, so it can prefer the ordinary grid
//     where the strided passes gain).
// The first two are searched jointly, then each pass's run length is halved
// in turn and kept where it is faster, then the three persistent settings are
// tried on the result; the three fastest choices are finally timed again,
// interleaved and longer, and the fastest of that round is kept.  The device
// is first warmed up by three applies; each candidate then runs once to warm
// up and 10 times between HIP events (3 timed runs left the choice to noise
// of about 2 %), the final three 2 x 30 times.
//
// Cache: a JSON array, one object per line,
//   {"key": "<arch>|cu=<CUs>|v=3|n=<n>|P=<P>|form=<f>|prec=<p>|nrhs=<b>|max_rhs=<m>",
//    "chunk": c, "kmul_w": w, "half_runs": r, "persist": q, "ms_per_rhs": t}
// read before timing (a hit skips it) and rewritten with the new entry after.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"
#include "tune.h"

namespace ls {

namespace {

std::string tune_key(const ApplyPlan& ap, int nrhs, ls_prec prec) {
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s|cu=%d|v=3|n=%d|P=%d|form=%d|prec=%d|nrhs=%d|max_rhs=%d", arch.c_str(), cus,
                ap.n, ap.P, ap.form, (int)prec, nrhs, ap.max_rhs);
  return buf;
}

struct Entry {
  std::string key;
  ApplyTune t;
  double ms = 0.0;
};

bool parse_int_field(const std::string& line, const char* name, int* v) {
  const std::string pat = std::string("\"") + name + "\":";
  const size_t p = line.find(pat);
  if (p == std::string::npos) return false;
  return std::sscanf(line.c_str() + p + pat.size(), " %d", v) == 1;
}

std::vector<Entry> read_cache(const std::string& path) {
  std::vector<Entry> out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t k = line.find("\"key\": \"");
    if (k == std::string::npos) continue;
    const size_t k0 = k + 8, k1 = line.find('"', k0);
    if (k1 == std::string::npos) continue;
    Entry e;
    e.key = line.substr(k0, k1 - k0);
    if (!parse_int_field(line, "chunk", &e.t.chunk) || !parse_int_field(line, "kmul_w", &e.t.kmul_w) ||
        !parse_int_field(line, "half_runs", &e.t.half_runs) || !parse_int_field(line, "persist", &e.t.persist))
      continue;
    const size_t t = line.find("\"ms_per_rhs\":");
    if (t != std::string::npos) std::sscanf(line.c_str() + t + 13, " %lf", &e.ms);
    out.push_back(e);
  }
  return out;
}

bool write_cache(const std::string& path, const std::vector<Entry>& es) {
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return false;
    f << "[\n";
    for (size_t i = 0; i < es.size(); ++i) {
      char buf[512];
      std::snprintf(buf, sizeof buf,
                    "{\"key\": \"%s\", \"chunk\": %d, \"kmul_w\": %d, \"half_runs\": %d, \"persist\": %d, "
                    "\"ms_per_rhs\": %.6g}%s\n",
                    es[i].key.c_str(), es[i].t.chunk, es[i].t.kmul_w, es[i].t.half_runs, es[i].t.persist, es[i].ms,
                    i + 1 < es.size() ? "," : "");
      f << buf;
    }
    f << "]\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

// average ms of one batched apply under the plan's current choice (one
// untimed apply first, then reps between events)
ls_status time_apply(ApplyPlan& ap, const void* x, void* y, int nrhs, ls_prec prec, hipStream_t s,
                     hipEvent_t e0, hipEvent_t e1, double* ms, int kReps = 10) {
  LS_TRY(apply_batched(ap, x, y, nrhs, prec, s));
  LS_HIP(hipEventRecord(e0, s));
  for (int r = 0; r < kReps; ++r) LS_TRY(apply_batched(ap, x, y, nrhs, prec, s));
  LS_HIP(hipEventRecord(e1, s));
  LS_HIP(hipEventSynchronize(e1));
  float t = 0.f;
  LS_HIP(hipEventElapsedTime(&t, e0, e1));
  *ms = (double)t / kReps;
  return LS_OK;
}

}  // namespace

ls_status apply_tune(ApplyPlan& ap, const std::string& cache, int nrhs, ls_prec prec, hipStream_t s,
                     TuneOutcome* out) {
  if (nrhs < 1) return LS_EINVAL;
  if (prec != LS_C128 && prec != LS_C64 && prec != LS_MIXED) return LS_EINVAL;
  if (ap.form != 0) return LS_ESTATE;       // the paper's form has a single launch choice
  TuneOutcome res;
  const std::string key = tune_key(ap, nrhs, prec);
  std::vector<Entry> entries;
  if (!cache.empty()) {
    entries = read_cache(cache);
    for (const Entry& e : entries)
      if (e.key == key && e.t.chunk >= 1 && e.t.chunk <= ap.max_rhs && e.t.kmul_w >= 1 && e.t.half_runs >= 0 &&
          e.t.half_runs <= 15 && e.t.persist >= 0 && e.t.persist <= 3) {
        ap.tune[prec] = e.t;
        res.t = e.t;
        res.ms_per_rhs = e.ms;
        res.from_cache = 1;
        if (out) *out = res;
        return LS_OK;
      }
  }
  const size_t es = (prec == LS_C64) ? 8 : 16;
  const size_t bytes = (size_t)nrhs * 3 * ap.n * ap.n * ap.n * es;
  DevBuf x, y;
  LS_TRY(x.alloc(bytes));
  LS_TRY(y.alloc(bytes));
  LS_HIP(hipMemsetAsync(x.p, 0x3c, bytes, s));     // small finite values in either precision
  hipEvent_t e0, e1;
  LS_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return LS_EHIP;
  }
  const ApplyTune saved = ap.tune[prec];
  std::vector<int> chunks;
  const int cmax = std::min(nrhs, ap.max_rhs);
  for (int c = 1; c < cmax; c *= 2) chunks.push_back(c);
  chunks.push_back(cmax);
  const std::vector<int> teams = kmul_team_choices(ap);
  ls_status st = LS_OK;
  double best = 1e300;
  ApplyTune pick = saved;
  // the default choice first, for reference, after warming the device up
  ap.tune[prec] = ApplyTune{};
  for (int r = 0; r < 3 && st == LS_OK; ++r) st = apply_batched(ap, x.p, y.p, nrhs, prec, s);
  if (st != LS_OK) {
    ap.tune[prec] = saved;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
  }
  st = time_apply(ap, x.p, y.p, nrhs, prec, s, e0, e1, &res.ms_default_per_rhs);
  res.ms_default_per_rhs /= nrhs;
  std::vector<std::pair<double, ApplyTune>> tried;
  auto trial = [&](const ApplyTune& t) {
    if (st != LS_OK) return;
    ap.tune[prec] = t;
    double ms = 0.0;
    st = time_apply(ap, x.p, y.p, nrhs, prec, s, e0, e1, &ms);
    ++res.n_tried;
    if (st == LS_OK) tried.push_back({ms, t});
    if (st == LS_OK && ms < best) {
      best = ms;
      pick = t;
    }
  };
  // 1. rhs per launch set x pass-3 teams
  for (size_t ci = 0; ci < chunks.size(); ++ci)
    for (size_t wi = 0; wi < teams.size(); ++wi) {
      if (teams[wi] > chunks[ci]) continue;       // a team needs its own right-hand side
      ApplyTune t;
      t.chunk = chunks[ci];
      t.kmul_w = teams[wi];
      trial(t);
    }
  // 2. half runs, one strided pass at a time
  for (int bit = 1; bit <= 8; bit <<= 1) {
    ApplyTune t = pick;
    t.half_runs |= bit;
    trial(t);
  }
  // 3. persistent launches: strided passes, pass 3, both
  {
    const ApplyTune base = pick;
    for (int q = 1; q <= 3; ++q) {
      ApplyTune t = base;
      t.persist = q;
      trial(t);
    }
  }
  // 4. the three fastest again, interleaved over two rounds of 3 x the reps:
  // the candidates differ by about 1 %, as much as the drift of the device
  // clock over the search
  if (st == LS_OK && tried.size() > 1) {
    std::stable_sort(tried.begin(), tried.end(),
                     [](const std::pair<double, ApplyTune>& a, const std::pair<double, ApplyTune>& b) {
                       return a.first < b.first;
                     });
    const size_t nf = std::min<size_t>(3, tried.size());
    std::vector<double> tot(nf, 0.0);
    for (int round = 0; round < 2 && st == LS_OK; ++round)
      for (size_t i = 0; i < nf && st == LS_OK; ++i) {
        ap.tune[prec] = tried[i].second;
        double ms = 0.0;
        st = time_apply(ap, x.p, y.p, nrhs, prec, s, e0, e1, &ms, 30);
        tot[i] += ms;
      }
    if (st == LS_OK) {
      const size_t bi = std::min_element(tot.begin(), tot.end()) - tot.begin();
      pick = tried[bi].second;
      best = tot[bi] / 2;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != LS_OK) {
    ap.tune[prec] = saved;
    return st;
  }
  ap.tune[prec] = pick;
  res.t = pick;
  res.ms_per_rhs = best / nrhs;
  if (!cache.empty()) {
    Entry e;
    e.key = key;
    e.t = pick;
    e.ms = res.ms_per_rhs;
    entries.push_back(e);
    if (!write_cache(cache, entries)) res.cache_write_failed = 1;
  }
  if (out) *out = res;
  return LS_OK;
}

}  // namespace ls
