// Autotuner for the launch shape and work split of the searches.
//
// The paper tunes its CPU partition factor lambda (Algorithm 5, Eq. 4) and
// the alpha/beta switch by grid search ("Parameter Tuning").  On the GPU the
// knobs that decide speed, and never the result, are: workgroup size and
// workgroups per compute unit of the persistent search, the row length up to
// which a bottom-up row is scanned by one lane rather than a whole wave, the
// number of edge-balanced bottom-up ranges per workgroup (the work-stealing
// grain), the top-down chunk length of the edge-balanced expansion, and how
// the internal arrays are cleared between searches.  The tuner times
// candidates by coordinate descent from the built-in defaults (sweeps over
// the parameters repeated until one moves nothing, at most three) and accepts a
// candidate only if its depth and parent arrays equal, entry for entry, those
// of the defaults on the same roots.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/rbfs.h"
#include "common.h"
#include "graph.h"
#include "handles.h"

namespace rbfs {

// The defaults are the tuner's winners on the Kronecker graphs of scale 26
// (single-root and 64-root searches); scales 27 and 28 move only bu_grain.
rbfs_tuning_t default_tuning(int kind) {
  rbfs_tuning_t t;
  t.block = 1024;
  t.per_cu = 1;
  t.lane_row = kind == RBFS_TUNE_BATCH ? 64 : 256;
  t.bu_grain = kind == RBFS_TUNE_BATCH ? 128 : 64;
  t.td_chunk = kTdK * 1024;
  t.reset = 0;
  return t;
}

bool tuning_valid(int kind, const rbfs_tuning_t& t, std::string* why) {
  const char* bad = nullptr;
  if (kind != RBFS_TUNE_SINGLE && kind != RBFS_TUNE_BATCH) bad = "unknown kind";
  else if (t.block != 1024 && !(kind == RBFS_TUNE_SINGLE && t.block == 256))
    bad = "block must be 1024 (or 256 for single-root searches)";
  else if (t.per_cu < 1 || t.per_cu > 4) bad = "per_cu outside [1, 4]";
  else if (t.lane_row < 1 || t.lane_row > 4096) bad = "lane_row outside [1, 4096]";
  else if (t.bu_grain < 1 || t.bu_grain > 1024) bad = "bu_grain outside [1, 1024]";
  else if (t.td_chunk < 256 || t.td_chunk > kTdK * t.block || (t.td_chunk & (t.td_chunk - 1)))
    bad = "td_chunk must be a power of two in [256, 4 * block]";
  else if (t.reset != 0 && t.reset != 1) bad = "reset must be 0 or 1";
  if (bad && why) *why = bad;
  return bad == nullptr;
}

namespace {

// Bound p of the ranges: the first word whose first vertex starts at or past
// adjacency entry p * target (the row offsets are the degree prefix sum).
__global__ void edge_range_kernel(const int64_t* off, int64_t n_sweep, int64_t target,
                                  int64_t nparts, int32_t* bounds) {
  const int64_t W = ceil_div(n_sweep, kWave);
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p <= nparts;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t want = p * target;
    int64_t lo = 0, hi = n_sweep;  // first vertex with off[v] >= want
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (off[mid] < want) lo = mid + 1; else hi = mid;
    }
    int64_t w = ceil_div(lo, kWave);
    if (p == nparts || w > W) w = W;
    bounds[p] = (int32_t)w;
  }
}

// Adds the number of positions where a and b differ to *cnt.
__global__ void count_diff_kernel(const int32_t* a, const int32_t* b, int64_t n,
                                  unsigned long long* cnt) {
  int64_t c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    c += (a[i] != b[i]) ? 1 : 0;
  c = wave_sum(c);
  if (lane_id() == 0 && c) atomicAdd(cnt, (unsigned long long)c);
}

}  // namespace

#define TUNE_CHECK(x)                                                           \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      set_error(std::string("tune: ") + #x + ": " + hipGetErrorString(e_));     \
      return e_ == hipErrorOutOfMemory ? RBFS_E_NOMEM : RBFS_E_DEVICE;          \
    }                                                                           \
  } while (0)

int build_edge_ranges(const int64_t* off, int64_t n_sweep, int64_t nnz, int64_t nparts_want,
                      int64_t min_words, int32_t** bounds, int32_t* n_part, hipStream_t stream) {
  const int64_t W = ceil_div(n_sweep > 0 ? n_sweep : 1, kWave);
  const int64_t want = std::max<int64_t>(1, nparts_want);
  const int64_t target = std::max<int64_t>(2048, nnz / want + 1);
  const int64_t nparts_e = std::max<int64_t>(1, ceil_div(nnz, target));
  const int64_t max_words = std::max<int64_t>(min_words, W / want + 1);
  int32_t* d_b = nullptr;
  TUNE_CHECK(rbfs::dev_malloc(&d_b, sizeof(int32_t) * (nparts_e + 1)));
  const int64_t blocks = std::min<int64_t>(ceil_div(nparts_e + 1, 256), 1 << 20);
  hipLaunchKernelGGL(edge_range_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, off,
                     n_sweep, target, nparts_e, d_b);
  hipError_t e = hipGetLastError();
  std::vector<int32_t> hb(nparts_e + 1);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hb.data(), d_b, sizeof(int32_t) * (nparts_e + 1), hipMemcpyDeviceToHost,
                       stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  (void)rbfs::dev_free(d_b);
  TUNE_CHECK(e);
  // split ranges that span too many (nearly empty) words
  std::vector<int32_t> parts{0};
  for (int64_t p = 1; p <= nparts_e; ++p) {
    int32_t a = parts.back(), b = std::max(hb[p], a);
    while (b - a > max_words) {
      a += (int32_t)max_words;
      parts.push_back(a);
    }
    if (b > parts.back()) parts.push_back(b);
  }
  if (parts.back() != (int32_t)W) parts.push_back((int32_t)W);
  int32_t* d = nullptr;
  TUNE_CHECK(rbfs::dev_malloc(&d, sizeof(int32_t) * parts.size()));
  e = hipMemcpyAsync(d, parts.data(), sizeof(int32_t) * parts.size(), hipMemcpyHostToDevice,
                     stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) (void)rbfs::dev_free(d);
  TUNE_CHECK(e);
  *bounds = d;
  *n_part = (int32_t)parts.size() - 1;
  return 0;
}

}  // namespace rbfs

using rbfs::Graph;
using rbfs::set_error;

namespace {

// Device buffers of one tuning session, freed on every exit path.
struct TuneBuffers {
  int32_t* ref_d = nullptr;
  int32_t* ref_p = nullptr;
  int32_t* cand_d = nullptr;
  int32_t* cand_p = nullptr;
  unsigned long long* diff = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~TuneBuffers() {
    void* ps[] = {ref_d, ref_p, cand_d, cand_p, diff};
    for (void* p : ps)
      if (p) (void)rbfs::dev_free(p);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

int hip_fail(const char* what, hipError_t e) {
  set_error(std::string("tune: ") + what + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? RBFS_E_NOMEM : RBFS_E_DEVICE;
}

// Counts the entries where a and b (n each) differ; synchronises.
int count_diff(TuneBuffers& B, const int32_t* a, const int32_t* b, int64_t n,
               hipStream_t stream, int64_t* out) {
  hipError_t e = hipMemsetAsync(B.diff, 0, sizeof(unsigned long long), stream);
  if (e != hipSuccess) return hip_fail("clear counter", e);
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(rbfs::ceil_div(n, 256), 8192));
  if (n > 0)
    hipLaunchKernelGGL(rbfs::count_diff_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, a,
                       b, n, B.diff);
  e = hipGetLastError();
  unsigned long long h = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&h, B.diff, sizeof(h), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail("compare outputs", e);
  *out = (int64_t)h;
  return 0;
}

// One dimension of the coordinate descent: the values a parameter may take.
struct Dim {
  const char* name;
  std::vector<std::pair<int, int>> values;  // (first, second) field values
  void (*set)(rbfs_tuning_t&, std::pair<int, int>);
};

void set_shape(rbfs_tuning_t& t, std::pair<int, int> v) {
  t.block = v.first;
  t.per_cu = v.second;
  t.td_chunk = std::min(t.td_chunk, rbfs::kTdK * t.block);  // a chunk fits the block's LDS
}
void set_lane_row(rbfs_tuning_t& t, std::pair<int, int> v) { t.lane_row = v.first; }
void set_grain(rbfs_tuning_t& t, std::pair<int, int> v) { t.bu_grain = v.first; }
void set_chunk(rbfs_tuning_t& t, std::pair<int, int> v) { t.td_chunk = v.first; }
void set_reset(rbfs_tuning_t& t, std::pair<int, int> v) { t.reset = v.first; }

bool same_tuning(const rbfs_tuning_t& a, const rbfs_tuning_t& b) {
  return memcmp(&a, &b, sizeof(a)) == 0;
}

// Candidate evaluation: apply(t) sets the parameters, check() runs every
// root once into the candidate buffers and returns the mismatch count,
// timed(reps) runs the timed repetitions and returns mean ms per call.
template <class Apply, class Check, class Timed>
int descend(int kind, const std::vector<Dim>& dims, rbfs_tuning_t start, Apply apply, Check check,
            Timed timed, int reps, rbfs_tuning_t* best_out, rbfs_tune_record_t* records,
            int32_t cap, int32_t* count, bool* any_mismatch) {
  int nrec = 0;
  auto evaluate = [&](const rbfs_tuning_t& t, float* ms, int64_t* mism) -> int {
    int rc = apply(t);
    if (!rc) rc = check(mism);
    if (!rc) rc = timed(reps, ms);
    if (rc) return rc;
    if (records && nrec < cap) {
      records[nrec].tuning = t;
      records[nrec].ms = *ms;
      records[nrec].mismatches = (int32_t)std::min<int64_t>(*mism, 0x7FFFFFFF);
    }
    ++nrec;
    if (*mism) *any_mismatch = true;
    return 0;
  };
  rbfs_tuning_t best = start;
  float best_ms = 0.f;
  int64_t mism = 0;
  int rc = evaluate(best, &best_ms, &mism);
  if (rc) return rc;
  // sweeps over the dimensions until one moves nothing: a later dimension's
  // move can change which value of an earlier one is best
  constexpr int kMaxSweeps = 3;
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    bool moved = false;
    for (const Dim& d : dims) {
      rbfs_tuning_t dim_best = best;
      float dim_ms = best_ms;
      for (const auto& v : d.values) {
        rbfs_tuning_t t = best;
        d.set(t, v);
        if (same_tuning(t, best) || !rbfs::tuning_valid(kind, t, nullptr)) continue;
        float ms = 0.f;
        rc = evaluate(t, &ms, &mism);
        if (rc) return rc;
        if (mism == 0 && ms < 0.99f * dim_ms) {
          dim_best = t;
          dim_ms = ms;
        }
      }
      if (!same_tuning(dim_best, best)) {
        // re-time the winner against the incumbent once more before moving
        float ms_new = 0.f, ms_old = 0.f;
        rc = apply(dim_best);
        if (!rc) rc = timed(reps, &ms_new);
        if (!rc) rc = apply(best);
        if (!rc) rc = timed(reps, &ms_old);
        if (rc) return rc;
        if (ms_new < 0.99f * ms_old) {
          best = dim_best;
          best_ms = ms_new;
          moved = true;
        } else {
          best_ms = ms_old;
        }
      }
    }
    if (!moved) break;
  }
  rc = apply(best);
  if (rc) return rc;
  if (best_out) *best_out = best;
  if (count) *count = std::min(nrec, cap > 0 ? cap : 0);
  return 0;
}

int valid_kind_args(int32_t kind, const int32_t* roots, int32_t k, int32_t reps, int32_t cap,
                    const char* fn) {
  if ((kind != RBFS_TUNE_SINGLE && kind != RBFS_TUNE_BATCH) || !roots || k < 1 || k > 64 ||
      reps < 1 || cap < 0) {
    set_error(std::string(fn) + ": bad arguments");
    return RBFS_E_INVAL;
  }
  return 0;
}

int apply_graph_tuning(Graph* g, int32_t kind, const rbfs_tuning_t& t, hipStream_t stream) {
  std::string why;
  if (!rbfs::tuning_valid(kind, t, &why)) {
    set_error("tuning: " + why);
    return RBFS_E_INVAL;
  }
  if (kind == RBFS_TUNE_SINGLE) {
    g->tune_single = t;
    return rbfs::bfs_apply_tuning(g, stream);
  }
  g->tune_batch = t;
  return g->ms ? rbfs::ms_apply_tuning(g->ms, t, stream) : 0;
}

}  // namespace

extern "C" {

int rbfs_tuning_default(int32_t kind, rbfs_tuning_t* t) {
  if (!t || (kind != RBFS_TUNE_SINGLE && kind != RBFS_TUNE_BATCH)) {
    set_error("rbfs_tuning_default: bad arguments");
    return RBFS_E_INVAL;
  }
  *t = rbfs::default_tuning(kind);
  return RBFS_OK;
}

int rbfs_graph_set_tuning(rbfs_graph_t* h, int32_t kind, const rbfs_tuning_t* t,
                          void* stream) {
  if (!h || !t) {
    set_error("rbfs_graph_set_tuning: NULL argument");
    return RBFS_E_INVAL;
  }
  if (hipSetDevice(h->g.device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return RBFS_E_DEVICE;
  }
  return apply_graph_tuning(&h->g, kind, *t, (hipStream_t)stream);
}

int rbfs_graph_get_tuning(const rbfs_graph_t* h, int32_t kind, rbfs_tuning_t* t) {
  if (!h || !t || (kind != RBFS_TUNE_SINGLE && kind != RBFS_TUNE_BATCH)) {
    set_error("rbfs_graph_get_tuning: bad arguments");
    return RBFS_E_INVAL;
  }
  *t = kind == RBFS_TUNE_SINGLE ? h->g.tune_single : h->g.tune_batch;
  return RBFS_OK;
}

int rbfs_tune(rbfs_graph_t* h, int32_t kind, const int32_t* roots, int32_t k, int32_t reps,
              const rbfs_opts_t* opts, rbfs_tuning_t* best, rbfs_tune_record_t* records,
              int32_t cap, int32_t* count, void* stream_) {
  if (!h) {
    set_error("rbfs_tune: NULL graph");
    return RBFS_E_INVAL;
  }
  int rc = valid_kind_args(kind, roots, k, reps, cap, "rbfs_tune");
  if (rc) return rc;
  if (count) *count = 0;
  Graph* g = &h->g;
  for (int32_t j = 0; j < k; ++j)
    if (roots[j] < 0 || roots[j] >= g->n) {
      set_error("rbfs_tune: root out of range");
      return RBFS_E_RANGE;
    }
  rbfs_opts_t o{};
  o.direction = RBFS_DIR_HEURISTIC;
  o.alpha = 14;
  o.beta = 24;
  o.output_space = RBFS_OUT_ORIGINAL;
  if (opts) {
    o = *opts;
    o.flags = 0;
    o.tune_profile = 0;
  }
  if (hipSetDevice(g->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return RBFS_E_DEVICE;
  }
  hipStream_t stream = (hipStream_t)stream_;
  const int64_t n = g->n > 0 ? g->n : 1;
  const int64_t cand_n = kind == RBFS_TUNE_SINGLE ? n : n * k;
  TuneBuffers B;
  hipError_t e = rbfs::dev_malloc(&B.ref_d, sizeof(int32_t) * n * k);
  if (e == hipSuccess) e = rbfs::dev_malloc(&B.ref_p, sizeof(int32_t) * n * k);
  if (e == hipSuccess) e = rbfs::dev_malloc(&B.cand_d, sizeof(int32_t) * cand_n);
  if (e == hipSuccess) e = rbfs::dev_malloc(&B.cand_p, sizeof(int32_t) * cand_n);
  if (e == hipSuccess) e = rbfs::dev_malloc(&B.diff, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipEventCreate(&B.e0);
  if (e == hipSuccess) e = hipEventCreate(&B.e1);
  if (e != hipSuccess) return hip_fail("allocate", e);

  auto run_all = [&](int32_t* d, int32_t* p, int64_t stride) -> int {
    if (kind == RBFS_TUNE_BATCH) return rbfs_bfs_batch(h, roots, k, d, p, &o, stream, nullptr);
    for (int32_t j = 0; j < k; ++j) {
      const int r = rbfs_bfs(h, roots[j], d + stride * j, p + stride * j, &o, stream, nullptr);
      if (r) return r;
    }
    return 0;
  };
  // reference outputs from the built-in defaults
  const rbfs_tuning_t def = rbfs::default_tuning(kind);
  rc = apply_graph_tuning(g, kind, def, stream);
  if (!rc) rc = run_all(B.ref_d, B.ref_p, n);
  if (!rc) rc = rbfs_graph_check(h, stream);
  if (rc) return rc;

  auto apply = [&](const rbfs_tuning_t& t) { return apply_graph_tuning(g, kind, t, stream); };
  auto check = [&](int64_t* mism) -> int {
    *mism = 0;
    for (int32_t j = 0; j < (kind == RBFS_TUNE_BATCH ? 1 : k); ++j) {
      int r = 0;
      if (kind == RBFS_TUNE_BATCH)
        r = rbfs_bfs_batch(h, roots, k, B.cand_d, B.cand_p, &o, stream, nullptr);
      else
        r = rbfs_bfs(h, roots[j], B.cand_d, B.cand_p, &o, stream, nullptr);
      if (!r) r = rbfs_graph_check(h, stream);
      if (r) return r;
      const int64_t off = kind == RBFS_TUNE_BATCH ? 0 : n * j;
      int64_t m1 = 0, m2 = 0;
      r = count_diff(B, B.cand_d, B.ref_d + off, cand_n, stream, &m1);
      if (!r) r = count_diff(B, B.cand_p, B.ref_p + off, cand_n, stream, &m2);
      if (r) return r;
      *mism += m1 + m2;
    }
    return 0;
  };
  auto timed = [&](int nrep, float* ms) -> int {
    hipError_t he = hipEventRecord(B.e0, stream);
    if (he != hipSuccess) return hip_fail("event", he);
    for (int r = 0; r < nrep; ++r) {
      const int rr = run_all(B.cand_d, B.cand_p, 0);
      if (rr) return rr;
    }
    he = hipEventRecord(B.e1, stream);
    if (he == hipSuccess) he = hipEventSynchronize(B.e1);
    float t = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&t, B.e0, B.e1);
    if (he != hipSuccess) return hip_fail("timing", he);
    *ms = t / (float)(nrep * (kind == RBFS_TUNE_BATCH ? 1 : k));
    return rbfs_graph_check(h, stream);
  };

  std::vector<Dim> dims;
  if (kind == RBFS_TUNE_SINGLE) {
    dims.push_back({"shape", {{1024, 1}, {1024, 2}, {256, 1}, {256, 2}, {256, 4}}, set_shape});
    dims.push_back({"lane_row", {{8, 0}, {16, 0}, {32, 0}, {64, 0}, {128, 0}, {256, 0}},
                    set_lane_row});
    dims.push_back({"bu_grain", {{8, 0}, {16, 0}, {32, 0}, {64, 0}, {128, 0}, {256, 0},
                                 {512, 0}, {1024, 0}},
                    set_grain});
    dims.push_back({"td_chunk", {{256, 0}, {512, 0}, {1024, 0}, {2048, 0}, {4096, 0}},
                    set_chunk});
    if (g->reordered && o.output_space == RBFS_OUT_ORIGINAL)
      dims.push_back({"reset", {{0, 0}, {1, 0}}, set_reset});
  } else {
    dims.push_back({"shape", {{1024, 1}, {1024, 2}}, set_shape});
    dims.push_back({"lane_row", {{8, 0}, {16, 0}, {32, 0}, {64, 0}, {128, 0}}, set_lane_row});
    dims.push_back({"bu_grain", {{4, 0}, {8, 0}, {16, 0}, {32, 0}, {64, 0}, {128, 0}},
                    set_grain});
  }
  // shapes that cannot be resident collapse onto smaller ones: drop them
  if (kind == RBFS_TUNE_SINGLE && g->bfs) {
    auto& v = dims[0].values;
    v.erase(std::remove_if(v.begin(), v.end(),
                           [&](std::pair<int, int> s) {
                             const int capc = s.first == 256 ? g->bfs->max_per_cu_256
                                                             : g->bfs->max_per_cu;
                             return s.second > capc;
                           }),
            v.end());
  } else if (kind == RBFS_TUNE_BATCH && g->ms) {
    auto& v = dims[0].values;
    v.erase(std::remove_if(v.begin(), v.end(),
                           [&](std::pair<int, int> s) { return s.second > g->ms->max_per_cu; }),
            v.end());
  }
  bool mismatch = false;
  rc = descend(kind, dims, def, apply, check, timed, reps, best, records, cap, count, &mismatch);
  if (rc) return rc;
  if (mismatch) {
    set_error("rbfs_tune: a candidate's outputs differ from the reference (see records)");
    return RBFS_E_DEVICE;
  }
  return RBFS_OK;
}

int rbfs_multi_set_tuning(rbfs_multi_t* m, const rbfs_tuning_t* t, void* stream_) {
  if (!m || !t) {
    set_error("rbfs_multi_set_tuning: NULL argument");
    return RBFS_E_INVAL;
  }
  std::string why;
  if (!rbfs::tuning_valid(RBFS_TUNE_BATCH, *t, &why)) {
    set_error("tuning: " + why);
    return RBFS_E_INVAL;
  }
  if (hipSetDevice(m->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return RBFS_E_DEVICE;
  }
  hipStream_t stream = stream_ ? (hipStream_t)stream_ : m->own_stream;
  return rbfs::ms_apply_tuning(&m->eng, *t, stream);
}

int rbfs_multi_get_tuning(const rbfs_multi_t* m, rbfs_tuning_t* t) {
  if (!m || !t) {
    set_error("rbfs_multi_get_tuning: NULL argument");
    return RBFS_E_INVAL;
  }
  *t = m->eng.tune;
  return RBFS_OK;
}

int rbfs_multi_tune(rbfs_multi_t* m, const int32_t* roots, int32_t k, int32_t reps,
                    rbfs_tuning_t* best, rbfs_tune_record_t* records, int32_t cap,
                    int32_t* count, void* stream_) {
  if (!m) {
    set_error("rbfs_multi_tune: NULL handle");
    return RBFS_E_INVAL;
  }
  int rc = valid_kind_args(RBFS_TUNE_BATCH, roots, k, reps, cap, "rbfs_multi_tune");
  if (rc) return rc;
  if (count) *count = 0;
  const int G = (int)m->gs.size();
  int64_t total = 0;
  for (int i = 0; i < G; ++i) {
    for (int32_t j = 0; j < k; ++j) {
      const int32_t r = roots[(int64_t)i * k + j];
      if (r < 0 || r >= m->gs[i]->n) {
        set_error("rbfs_multi_tune: root out of range");
        return RBFS_E_RANGE;
      }
    }
    total += m->gs[i]->n;
  }
  if (hipSetDevice(m->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return RBFS_E_DEVICE;
  }
  // a NULL stream runs the searches on the handle's own stream: time there
  hipStream_t stream = stream_ ? (hipStream_t)stream_ : m->own_stream;
  const int64_t out_n = std::max<int64_t>(1, total * k);
  TuneBuffers B;
  hipError_t e = rbfs::dev_malloc(&B.ref_d, sizeof(int32_t) * out_n);
  if (e == hipSuccess) e = rbfs::dev_malloc(&B.ref_p, sizeof(int32_t) * out_n);
  if (e == hipSuccess) e = rbfs::dev_malloc(&B.cand_d, sizeof(int32_t) * out_n);
  if (e == hipSuccess) e = rbfs::dev_malloc(&B.cand_p, sizeof(int32_t) * out_n);
  if (e == hipSuccess) e = rbfs::dev_malloc(&B.diff, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipEventCreate(&B.e0);
  if (e == hipSuccess) e = hipEventCreate(&B.e1);
  if (e != hipSuccess) return hip_fail("allocate", e);
  auto apply = [&](const rbfs_tuning_t& t) { return rbfs_multi_set_tuning(m, &t, stream); };
  const rbfs_tuning_t def = rbfs::default_tuning(RBFS_TUNE_BATCH);
  rc = apply(def);
  if (!rc) rc = rbfs_bfs_multi(m, roots, k, B.ref_d, B.ref_p, nullptr, stream, nullptr);
  if (rc) return rc;
  auto check = [&](int64_t* mism) -> int {
    int r = rbfs_bfs_multi(m, roots, k, B.cand_d, B.cand_p, nullptr, stream, nullptr);
    int64_t m1 = 0, m2 = 0;
    if (!r) r = count_diff(B, B.cand_d, B.ref_d, total * k, stream, &m1);
    if (!r) r = count_diff(B, B.cand_p, B.ref_p, total * k, stream, &m2);
    *mism = m1 + m2;
    return r;
  };
  auto timed = [&](int nrep, float* ms) -> int {
    hipError_t he = hipEventRecord(B.e0, stream);
    if (he != hipSuccess) return hip_fail("event", he);
    for (int r = 0; r < nrep; ++r) {
      const int rr = rbfs_bfs_multi(m, roots, k, B.cand_d, B.cand_p, nullptr, stream, nullptr);
      if (rr) return rr;
    }
    he = hipEventRecord(B.e1, stream);
    if (he == hipSuccess) he = hipEventSynchronize(B.e1);
    float t = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&t, B.e0, B.e1);
    if (he != hipSuccess) return hip_fail("timing", he);
    *ms = t / (float)nrep;
    return 0;
  };
  std::vector<Dim> dims;
  dims.push_back({"shape", {{1024, 1}, {1024, 2}}, set_shape});
  dims.push_back({"lane_row", {{8, 0}, {16, 0}, {32, 0}, {64, 0}, {128, 0}}, set_lane_row});
  dims.push_back({"bu_grain", {{4, 0}, {8, 0}, {16, 0}, {32, 0}, {64, 0}, {128, 0}},
                  set_grain});
  auto& v = dims[0].values;
  v.erase(std::remove_if(v.begin(), v.end(),
                         [&](std::pair<int, int> s) { return s.second > m->eng.max_per_cu; }),
          v.end());
  bool mismatch = false;
  rc = descend(RBFS_TUNE_BATCH, dims, def, apply, check, timed, reps, best, records, cap, count,
               &mismatch);
  if (rc) return rc;
  if (mismatch) {
    set_error("rbfs_multi_tune: a candidate's outputs differ from the reference (see records)");
    return RBFS_E_DEVICE;
  }
  return RBFS_OK;
}

}  // extern "C"
