// Reverse Cuthill-McKee relabelling on the GPU (Algorithm 3, section 3.2),
// equal to the sequential algorithm label for label.
//
// Sequential Algorithm 3 labels vertices in queue order: a component starts
// at its unvisited vertex of least (degree, id) and every processed vertex
// appends its unvisited neighbours in increasing (degree, id) order.  Since a
// whole BFS level is labelled before any vertex of it is processed, a vertex
// w of level L+1 is appended by its level-L neighbour with the smallest
// label, and level L+1 is ordered by (that label, degree(w), id(w)).
// Components are explored in increasing order of their start key and each
// occupies one contiguous label range.  The GPU pass therefore:
//   1. ranks V+ by (degree, id) (radix sort of degree << b | id);
//   2. finds connected components by union-find in rank space, always
//      linking the larger root under the smaller, so each root is the
//      component's minimum-rank vertex, i.e. its start;
//   3. gives each component the label base = number of vertices in
//      components with a smaller start rank (scan of component sizes);
//   4. runs Cuthill-McKee level by level for all components at once: every
//      unlabelled neighbour w of the current level takes the minimum label of
//      its level neighbours (atomicMin), the new level is sorted by
//      (that label, rank(w)), and labels are handed out per component in that
//      order;
//   5. reverses the labels over V+, appends the isolated vertices in
//      increasing id, and rebuilds the CSR in the new labels with every row
//      ascending (the relabelled rows transposed by one stable sort on the
//      old column, then each group copied to its new row).
//
// Partial RCM (section 4.6) reorders only the first `keep` vertices of the
// Cuthill-McKee sequence: they take labels [0, keep) in reverse sequence
// order, the other non-isolated vertices follow in increasing id, isolated
// vertices last.  A vertex's sequence position depends only on vertices
// of smaller position (its level, the labels of the level before, the ranks
// of its level), so the level loop seeds only the components that start
// below `keep` and expands only vertices labelled below `keep`: every label
// below `keep` comes out as in the full pass, and a vertex labelled later
// (possibly at a wrong level, when its true parents were not expanded)
// always gets a label of at least `keep`, because its component's next free
// label has passed `keep` by then.  Within a level the labels rise with the
// sorted position, so the vertices to expand next form a prefix.
#include <hip/hip_runtime.h>

#include <stdlib.h>

#include <algorithm>
#include <string>
#include <vector>

#include "common.h"
#include "expand.h"
#include "graph.h"
#include "prim.h"

namespace rbfs {
namespace {

constexpr uint32_t kUnset = 0xFFFFFFFFu;

int grid_for(int64_t work) {
  int64_t b = ceil_div(work, kBlock);
  if (b < 1) b = 1;
  if (b > (1 << 20)) b = 1 << 20;
  return (int)b;
}

// Grid of a grid-stride kernel that folds a shared counter once per wave:
// few enough waves that the same-address atomics stay cheap (each costs
// about 10 ns, in series), enough workgroups to fill the GPU.
int grid_folding(int64_t work) {
  const int b = grid_for(work);
  return b < kFoldBlocks ? b : kFoldBlocks;
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
       i += (int64_t)gridDim.x * blockDim.x)

__global__ void deg_kernel(const int64_t* off, int64_t n, int32_t* deg, int32_t* nz,
                           unsigned long long* maxdeg) {
  int64_t dmax = 0;
  GRID_STRIDE(v, n) {
    const int64_t d = off[v + 1] - off[v];
    deg[v] = (int32_t)d;
    nz[v] = d > 0 ? 1 : 0;
    dmax = d > dmax ? d : dmax;
  }
  // one atomic per wave on the shared maximum
  dmax = wave_max(dmax);
  if (lane_id() == 0 && dmax > 0) atomicMax(maxdeg, (unsigned long long)dmax);
}

__global__ void deg_keys_kernel(const int32_t* deg, const int64_t* pos_nz, int64_t n, int bv,
                                uint64_t* keys) {
  GRID_STRIDE(v, n) {
    if (deg[v] > 0) keys[pos_nz[v]] = ((uint64_t)deg[v] << bv) | (uint64_t)v;
  }
}

__global__ void vplus_kernel(const uint64_t* keys, int64_t nplus, int bv, int32_t* vplus,
                             int32_t* rank, int32_t* ccp) {
  const uint64_t mask = (1ull << bv) - 1ull;
  GRID_STRIDE(k, nplus) {
    const int32_t v = (int32_t)(keys[k] & mask);
    vplus[k] = v;
    rank[v] = (int32_t)k;
    ccp[k] = (int32_t)k;
  }
}

// Union-find with the larger root linked under the smaller root (hooking as
// in ECL-CC, Jaiganesh and Burtscher, HPDC 2018).  Parent pointers only ever
// decrease, so racy reads are safe.
__device__ __forceinline__ int32_t uf_find(int32_t* p, int32_t x) {
  int32_t cur = __hip_atomic_load(&p[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (cur != x) {
    int32_t prev = x;
    int32_t next;
    while (cur > (next = __hip_atomic_load(&p[cur], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT))) {
      __hip_atomic_store(&p[prev], next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      prev = cur;
      cur = next;
    }
  }
  return cur;
}

__device__ __forceinline__ void uf_union(int32_t* p, int32_t a, int32_t b) {
  int32_t ra = uf_find(p, a);
  int32_t rb = uf_find(p, b);
  while (ra != rb) {
    if (ra < rb) {
      const int32_t old = atomicCAS(&p[rb], rb, ra);
      if (old == rb) break;
      rb = old;
    } else {
      const int32_t old = atomicCAS(&p[ra], ra, rb);
      if (old == ra) break;
      ra = old;
    }
  }
}

// Components in two passes, after Afforest (Sutton, Ben-Nun and Barak,
// IPDPS 2018).  The sampling pass links every vertex with its first
// kCcSample neighbours, which already joins most of a power-law graph into
// its giant component.  The full pass then takes every edge of the vertices
// that are not (yet) in the component of a chosen vertex `big`: an edge
// between a skipped vertex and a processed one is taken from the processed
// end, and two skipped vertices are already joined, so every edge is
// accounted for.  The hooking rule leaves the minimum rank as root whatever
// the order, so the result is that of a full pass over all edges.
constexpr int kCcSample = 2;

__global__ void cc_sample_kernel(const int64_t* off, const int32_t* cols, int64_t n,
                                 const int32_t* rank, int32_t* ccp) {
  GRID_STRIDE(v, n) {
    const int64_t b = off[v], e = off[v + 1];
    for (int64_t j = b; j < e && j < b + kCcSample; ++j) uf_union(ccp, rank[v], rank[cols[j]]);
  }
}

__global__ void cc_big_root_kernel(int32_t* ccp, int32_t big_rank, int32_t* big_root) {
  *big_root = uf_find(ccp, big_rank);
}

__global__ __launch_bounds__(kBlock) void cc_union_kernel(const int64_t* off, const int32_t* cols,
                                                          int64_t n, const int32_t* rank,
                                                          int32_t* ccp, const int32_t* big_root) {
  const int64_t nwords = ceil_div(n, kWave);
  const int64_t wstride = (int64_t)gridDim.x * kWavesPerBlock;
  const int32_t c = *big_root;
  const int l = lane_id();
  for (int64_t word = (int64_t)blockIdx.x * kWavesPerBlock + wave_id(); word < nwords;
       word += wstride) {
    const int64_t v = word * kWave + l;
    int64_t b = 0, e = 0;
    int32_t rv = 0;
    if (v < n) {
      b = off[v];
      e = off[v + 1];
      if (e > b) {
        rv = rank[v];
        if (uf_find(ccp, rv) == c) e = b;  // in the big component: skipped
      }
    }
    // rows of at most kLaneRow entries by their own lane, longer by the wave
    const bool big_row = (e - b) > kLaneRow;
    if (!big_row)
      for (int64_t j = b; j < e; ++j) uf_union(ccp, rv, rank[cols[j]]);
    uint64_t hubs = ballot(big_row);
    while (hubs) {
      const int h = ffs64(hubs);
      hubs &= hubs - 1;
      const int64_t hb = shfl(b, h), he = shfl(e, h);
      const int32_t hr = shfl(rv, h);
      for (int64_t j = hb + l; j < he; j += kWave) uf_union(ccp, hr, rank[cols[j]]);
    }
  }
}

// Final root of every rank and the component sizes.  One component usually
// holds almost every vertex, so the size counts are aggregated per wave: the
// lanes holding the wave's running root add to a register, flushed with one
// atomic when the root changes and at the end, instead of one same-address
// atomic per vertex or per batch.
__global__ void cc_compress_kernel(int32_t* ccp, int64_t nplus, int32_t* csize) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int32_t run_root = -1;  // the same in every lane
  int run_cnt = 0;        // lane 0's tally for run_root
  for (int64_t k0 = (int64_t)blockIdx.x * blockDim.x; k0 < nplus; k0 += stride) {
    const int64_t k = k0 + threadIdx.x;
    const bool act = k < nplus;
    int32_t p = -1;
    if (act) {
      int32_t x = (int32_t)k;
      p = ccp[x];
      while (p != x) {
        x = p;
        p = ccp[x];
      }
      ccp[k] = p;
    }
    const uint64_t am = ballot(act);
    if (am == 0) continue;
    const int32_t p0 = shfl(p, ffs64(am));
    if (p0 != run_root) {
      if (lane_id() == 0 && run_cnt > 0) atomicAdd(&csize[run_root], run_cnt);
      run_root = p0;
      run_cnt = 0;
    }
    const bool same = act && p == p0;
    const uint64_t sm = ballot(same);
    if (lane_id() == 0) run_cnt += popc64(sm);
    if (act && !same) atomicAdd(&csize[p], 1);
  }
  if (lane_id() == 0 && run_cnt > 0) atomicAdd(&csize[run_root], run_cnt);
}

// Component boundaries in the final (reversed) labelling.  Component roots
// taken in rank order have Cuthill-McKee label bases b_0 = 0 < b_1 < ... <
// b_K = nplus, and the whole sequence is reversed at the end, so component j
// occupies final labels [nplus - b_{j+1}, nplus - b_j).  With pos[k] = j for
// the root of rank k: bounds[K - j] = nplus - b_j, and bounds[0] = 0.
__global__ void comp_flag_kernel(const int32_t* ccp, int64_t nplus, int32_t* flag) {
  GRID_STRIDE(k, nplus) { flag[k] = ccp[k] == (int32_t)k ? 1 : 0; }
}

__global__ void comp_bounds_kernel(const int32_t* ccp, const int64_t* cbase, const int64_t* pos,
                                   int64_t nplus, int64_t K, int32_t* bounds) {
  GRID_STRIDE(k, nplus) {
    if (ccp[k] == (int32_t)k) bounds[K - pos[k]] = (int32_t)(nplus - cbase[k]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) bounds[0] = 0;
}

__device__ __forceinline__ void set_labelled(uint64_t* lbits, int32_t v) {
  atomicOr((unsigned long long*)&lbits[v >> 6], 1ull << (v & 63));
}

__global__ void cm_roots_kernel(const int32_t* ccp, const int64_t* cbase, const int32_t* vplus,
                                int64_t nplus, int64_t keep, int32_t* label, uint64_t* lbits,
                                int32_t* nextfree, int32_t* front, int32_t* front_count) {
  GRID_STRIDE(k, nplus) {
    if (ccp[k] == (int32_t)k && cbase[k] < keep) {
      const int32_t v = vplus[k];
      label[v] = (int32_t)cbase[k];
      set_labelled(lbits, v);
      nextfree[k] = (int32_t)cbase[k] + 1;
      const int pos = atomicAdd(front_count, 1);
      front[pos] = v;
    }
  }
}

__global__ void gather_deg_kernel(const int32_t* front, int64_t nf, const int32_t* deg,
                                  int32_t* out) {
  GRID_STRIDE(i, nf) { out[i] = deg[front[i]]; }
}

__global__ void mark_kernel(const int64_t* qe, int64_t nq, int32_t* chunk_pos, int64_t cap) {
  GRID_STRIDE(i, nq) { mark_chunks(chunk_pos, cap, qe[i], qe[i + 1] - qe[i], (int32_t)i); }
}

// CM expansion of one level: every unlabelled neighbour w takes the minimum
// label of its frontier neighbours; the first to touch w appends it.  Most
// edges of a level lead to labelled vertices; the labelled-vertex bitmap
// (n / 8 bytes, cache resident) rules them out without reading label[w].
// Four entries per thread are in flight at once.  The appended vertices are
// gathered in LDS and published a batch at a time, so the one global
// counter of the next level sees one atomic per batch instead of one per
// wave and round.
constexpr int kCmK = 4;
constexpr int kCmStage = 2048;  // LDS batch; a chunk appends at most kCmK * kBlock

__device__ __forceinline__ void cm_publish(const int32_t* s_new, int* s_cnt, int* s_base,
                                           int32_t* next, int32_t* next_count, int64_t next_cap,
                                           int* status) {
  const int cnt = *s_cnt;  // read after a barrier
  if (cnt > 0) {
    if (threadIdx.x == 0) *s_base = atomicAdd(next_count, cnt);
    __syncthreads();
    const int64_t base = *s_base;
    for (int i = threadIdx.x; i < cnt; i += kBlock) {
      if (base + i < next_cap) next[base + i] = s_new[i];
      else atomicOr(status, kStatusOverflow);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *s_cnt = 0;
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void cm_expand_kernel(
    const int32_t* front, const int64_t* qe, int64_t nq, int64_t E, const int32_t* chunk_pos,
    int64_t nchunks, const int64_t* off, const int32_t* cols, const int32_t* label,
    const uint64_t* lbits, uint32_t* plabel, int32_t* next, int32_t* next_count,
    int64_t next_cap, int* status) {
  __shared__ ChunkLdsB<kCmK * kBlock> s;
  __shared__ int32_t s_new[kCmStage];
  __shared__ int s_cnt, s_base;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const bool ok = expand_chunk_batch<kBlock, kCmK>(
        s, c, E, front, qe, nq, chunk_pos, nchunks, off, cols, kChunkShift,
        [&](const bool* act, const int32_t* u, const int32_t* w) {
      bool cand[kCmK], first[kCmK];
      uint32_t lu[kCmK], pl[kCmK];
#pragma unroll
      for (int r = 0; r < kCmK; ++r)
        cand[r] = act[r] && !((lbits[w[r] >> 6] >> (w[r] & 63)) & 1ull);
#pragma unroll
      for (int r = 0; r < kCmK; ++r) {
        lu[r] = cand[r] ? (uint32_t)label[u[r]] : 0u;
        pl[r] = cand[r] ? plabel[w[r]] : 0u;
      }
#pragma unroll
      for (int r = 0; r < kCmK; ++r) {
        // a stale read can only be larger: skip the atomic when w already
        // holds a label no larger than u's (then w was touched before)
        first[r] = false;
        if (cand[r] && pl[r] > lu[r]) first[r] = atomicMin(&plabel[w[r]], lu[r]) == kUnset;
      }
#pragma unroll
      for (int r = 0; r < kCmK; ++r) {
        const uint64_t m = ballot(first[r]);
        if (m) {
          const int leader = ffs64(m);
          int base = 0;
          if (lane_id() == leader) base = atomicAdd(&s_cnt, popc64(m));
          base = shfl(base, leader);
          if (first[r]) s_new[base + popc64(m & lanemask_lt())] = w[r];
        }
      }
    });
    if (!ok) {
      if (threadIdx.x == 0) atomicOr(status, kStatusBadInput);
      return;
    }
    // expand_chunk_batch ends with a barrier: s_cnt is final for the chunk
    if (s_cnt > kCmStage - kCmK * kBlock)
      cm_publish(s_new, &s_cnt, &s_base, next, next_count, next_cap, status);
  }
  cm_publish(s_new, &s_cnt, &s_base, next, next_count, next_cap, status);
}

__global__ void cm_keys_kernel(const int32_t* next, int64_t m, const uint32_t* plabel,
                               const int32_t* rank, int br, uint64_t* keys) {
  GRID_STRIDE(i, m) {
    const int32_t w = next[i];
    keys[i] = ((uint64_t)plabel[w] << br) | (uint64_t)rank[w];
  }
}

__global__ void cm_heads_kernel(const uint64_t* keys, int64_t m, int br, const int32_t* ccp,
                                int32_t* segstart) {
  const uint64_t mask = (1ull << br) - 1ull;
  GRID_STRIDE(i, m) {
    const int32_t c = ccp[keys[i] & mask];
    if (i == 0 || ccp[keys[i - 1] & mask] != c) segstart[c] = (int32_t)i;
  }
}

// Labels the sorted level and counts the entries labelled below `keep`
// (they lead the level: labels rise with the sorted position).
__global__ void cm_assign_kernel(const uint64_t* keys, int64_t m, int br, const int32_t* ccp,
                                 const int32_t* vplus, const int32_t* segstart,
                                 const int32_t* nextfree, int64_t keep, int32_t* label,
                                 uint64_t* lbits, int32_t* front, int32_t* below_keep) {
  const uint64_t mask = (1ull << br) - 1ull;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < m; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    bool low = false;
    if (i < m) {
      const int32_t r = (int32_t)(keys[i] & mask);
      const int32_t c = ccp[r];
      const int32_t w = vplus[r];
      const int32_t s = segstart[c];
      const int32_t lab = nextfree[c] + (int32_t)(i - s);
      label[w] = lab;
      set_labelled(lbits, w);
      front[i] = w;
      low = lab < keep;
    }
    const uint64_t bm = ballot(low);
    if (bm && lane_id() == ffs64(bm)) atomicAdd(below_keep, popc64(bm));
  }
}

// Separate launch: every thread of a segment must have read nextfree[c]
// before the segment's last element advances it.
__global__ void cm_advance_kernel(const uint64_t* keys, int64_t m, int br, const int32_t* ccp,
                                  const int32_t* segstart, int32_t* nextfree) {
  const uint64_t mask = (1ull << br) - 1ull;
  GRID_STRIDE(i, m) {
    const int32_t c = ccp[keys[i] & mask];
    if (i == m - 1 || ccp[keys[i + 1] & mask] != c) nextfree[c] += (int32_t)(i - segstart[c] + 1);
  }
}

// Vertices of V+ left out of a partial order (no label below keep).
__global__ void rest_flag_kernel(const int32_t* deg, const int32_t* label, int64_t n,
                                 int64_t keep, int32_t* flag) {
  GRID_STRIDE(v, n) {
    const int32_t l = label[v];
    flag[v] = (deg[v] > 0 && !(l >= 0 && l < keep)) ? 1 : 0;
  }
}

// Final labels: sequence position l < keep -> keep - 1 - l; the rest of V+
// (pos_rest: their exclusive prefix count in id order; null when keep = n+)
// -> keep + pos_rest; isolated -> n+ onwards in id order.
__global__ void perm_kernel(const int32_t* deg, const int32_t* label, const int64_t* pos_nz,
                            const int64_t* pos_rest, int64_t n, int64_t nplus, int64_t keep,
                            int32_t* perm, int32_t* iperm, int* status) {
  GRID_STRIDE(v, n) {
    int64_t p;
    if (deg[v] > 0) {
      const int32_t l = label[v];
      if (l >= 0 && l < keep) {
        p = keep - 1 - l;
      } else if (pos_rest) {
        p = keep + pos_rest[v];
      } else {
        atomicOr(status, kStatusBadInput);
        p = -1;
      }
    } else {
      p = nplus + (v - pos_nz[v]);
    }
    perm[v] = (int32_t)p;
    if (p >= 0 && p < n) iperm[p] = (int32_t)v;
  }
}

__global__ void newdeg_kernel(const int32_t* iperm, const int32_t* deg, int64_t n,
                              int32_t* newdeg) {
  GRID_STRIDE(i, n) { newdeg[i] = deg[iperm[i]]; }
}

// Relabelled CSR through one transpose.  Entry (v, w) becomes the pair
// (w, perm[v]) -- its old column and its new row -- stored in new-row order
// (row perm[v] at newoff[perm[v]]).  A stable sort on the old column alone
// groups the pairs by w, with the new labels of w's neighbours ascending
// inside each group; the groups come out in old order at the old offsets,
// and one copy of each group w to newoff[perm[w]] gives the new row
// perm[w], already sorted.  No per-entry relabelling gather is needed: the
// new labels come one per row.
__global__ __launch_bounds__(kBlock) void relabel_keys_kernel(const int64_t* off,
                                                              const int32_t* cols, int64_t n,
                                                              int64_t nnz, const int32_t* perm,
                                                              const int64_t* newoff,
                                                              uint64_t* keys, int* status) {
  const int64_t nwords = ceil_div(n, kWave);
  const int64_t wstride = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t word = (int64_t)blockIdx.x * kWavesPerBlock + wave_id(); word < nwords;
       word += wstride) {
    word_edges(off, cols, n, word, [&](int64_t v, int32_t w, int64_t e) {
      const int64_t r = perm[v];
      const int64_t pos = newoff[r] + (e - off[v]);
      if (pos >= 0 && pos < nnz) keys[pos] = ((uint64_t)(uint32_t)w << 32) | (uint64_t)r;
      else atomicOr(status, kStatusBadInput);
    });
  }
}

// Group w of the sorted pairs (entries [off[w], off[w + 1])) to new row
// perm[w]: rows of at most kLaneRow entries by one lane, longer ones by the
// whole wave.
__global__ __launch_bounds__(kBlock) void groups_to_rows_kernel(const int64_t* off, int64_t n,
                                                                int64_t nnz, const int32_t* perm,
                                                                const int64_t* newoff,
                                                                const uint64_t* keys,
                                                                int32_t* newcols, int* status) {
  const int64_t nwords = ceil_div(n, kWave);
  const int64_t wstride = (int64_t)gridDim.x * kWavesPerBlock;
  const int l = lane_id();
  for (int64_t word = (int64_t)blockIdx.x * kWavesPerBlock + wave_id(); word < nwords;
       word += wstride) {
    const int64_t w = word * kWave + l;
    int64_t b = 0, e = 0, dst = 0;
    if (w < n) {
      b = off[w];
      e = off[w + 1];
      if (e > b) {
        dst = newoff[perm[w]];
        if (dst < 0 || dst + (e - b) > nnz) {
          atomicOr(status, kStatusBadInput);
          e = b;
        }
      }
    }
    const bool big = (e - b) > kLaneRow;
    if (!big)
      for (int64_t j = b; j < e; ++j) newcols[dst + (j - b)] = (int32_t)(uint32_t)keys[j];
    uint64_t hubs = ballot(big);
    while (hubs) {
      const int h = ffs64(hubs);
      hubs &= hubs - 1;
      const int64_t hb = shfl(b, h), he = shfl(e, h), hd = shfl(dst, h);
      for (int64_t j = hb + l; j < he; j += kWave) newcols[hd + (j - hb)] = (int32_t)(uint32_t)keys[j];
    }
  }
}

// Batched relabel, for graphs whose whole-graph pair sort does not fit:
// new rows [k0, k1) at a time.  Entry j of new row k (the row of v =
// iperm[k]) gets the key ((k - k0) << bc) | perm[w] for its neighbour w, at
// its final position in the batch; one sort of the batch on those bits
// leaves every row ascending.  Rows of at most kLaneRow entries by one lane,
// longer ones by the whole wave.
__global__ __launch_bounds__(kBlock) void row_keys_kernel(const int64_t* off, const int32_t* cols,
                                                          const int32_t* iperm,
                                                          const int32_t* perm,
                                                          const int64_t* newoff, int64_t k0,
                                                          int64_t k1, int bc, uint64_t* keys,
                                                          int64_t cap, int* status) {
  const int64_t nw = ceil_div(k1 - k0, kWave);
  const int64_t wstride = (int64_t)gridDim.x * kWavesPerBlock;
  const int l = lane_id();
  const int64_t base = newoff[k0];
  for (int64_t word = (int64_t)blockIdx.x * kWavesPerBlock + wave_id(); word < nw;
       word += wstride) {
    const int64_t k = k0 + word * kWave + l;
    int64_t b = 0, e = 0, dst = 0;
    if (k < k1) {
      const int64_t v = iperm[k];
      b = off[v];
      e = off[v + 1];
      dst = newoff[k] - base;
      if (dst < 0 || dst + (e - b) > cap) {
        atomicOr(status, kStatusBadInput);
        e = b;
      }
    }
    const uint64_t hi = (uint64_t)(k - k0) << bc;
    const bool big = (e - b) > kLaneRow;
    if (!big)
      for (int64_t j = b; j < e; ++j) keys[dst + (j - b)] = hi | (uint32_t)perm[cols[j]];
    uint64_t hubs = ballot(big);
    while (hubs) {
      const int h = ffs64(hubs);
      hubs &= hubs - 1;
      const int64_t hb = shfl(b, h), he = shfl(e, h), hd = shfl(dst, h);
      const uint64_t hh = shfl(hi, h);
      for (int64_t j = hb + l; j < he; j += kWave) keys[hd + (j - hb)] = hh | (uint32_t)perm[cols[j]];
    }
  }
}

__global__ void keys_to_cols_kernel(const uint64_t* keys, int64_t m, int bc, int32_t* out) {
  const uint64_t mask = (1ull << bc) - 1ull;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int32_t)(keys[i] & mask);
}

// Batch bounds: kb[i] = the first row starting at or after entry i * per
// (i in [0, nb)), kb[nb] = n; eb[i] = newoff[kb[i]].
__global__ void batch_bounds_kernel(const int64_t* newoff, int64_t n, int64_t per, int64_t nb,
                                    int64_t* kb, int64_t* eb) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= nb;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t k = n;
    if (i < nb) {
      const int64_t want = i * per;
      int64_t lo = 0, hi = n;  // first k with newoff[k] >= want
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (newoff[mid] < want) lo = mid + 1;
        else hi = mid;
      }
      k = lo;
    }
    kb[i] = k;
    eb[i] = newoff[k];
  }
}

// Staged relabel (the old columns in host memory): old rows [v0, v1), whose
// columns st holds from entry e0 on, renamed by perm and copied to their new
// rows; each row is sorted afterwards.
__global__ __launch_bounds__(kBlock) void scatter_rows_kernel(const int64_t* off, int64_t v0,
                                                              int64_t v1, int64_t e0,
                                                              const int32_t* st,
                                                              const int32_t* perm,
                                                              const int64_t* newoff,
                                                              int32_t* newcols) {
  const int64_t nw = ceil_div(v1 - v0, kWave);
  const int64_t wstride = (int64_t)gridDim.x * kWavesPerBlock;
  const int l = lane_id();
  for (int64_t word = (int64_t)blockIdx.x * kWavesPerBlock + wave_id(); word < nw;
       word += wstride) {
    const int64_t v = v0 + word * kWave + l;
    int64_t b = 0, e = 0, dst = 0;
    if (v < v1) {
      b = off[v];
      e = off[v + 1];
      dst = newoff[perm[v]];
    }
    const bool big = (e - b) > kLaneRow;
    if (!big)
      for (int64_t j = b; j < e; ++j) newcols[dst + (j - b)] = perm[st[j - e0]];
    uint64_t hubs = ballot(big);
    while (hubs) {
      const int h = ffs64(hubs);
      hubs &= hubs - 1;
      const int64_t hb = shfl(b, h), he = shfl(e, h), hd = shfl(dst, h);
      for (int64_t j = hb + l; j < he; j += kWave) newcols[hd + (j - hb)] = perm[st[j - e0]];
    }
  }
}

// Keys of new rows [k0, k1) already renamed in place: ((k - k0) << bc) |
// column, at the entry's offset from the batch start.
__global__ __launch_bounds__(kBlock) void inplace_keys_kernel(const int64_t* newoff, int64_t k0,
                                                              int64_t k1, int bc,
                                                              const int32_t* newcols,
                                                              uint64_t* keys) {
  const int64_t nw = ceil_div(k1 - k0, kWave);
  const int64_t wstride = (int64_t)gridDim.x * kWavesPerBlock;
  const int l = lane_id();
  const int64_t base = newoff[k0];
  for (int64_t word = (int64_t)blockIdx.x * kWavesPerBlock + wave_id(); word < nw;
       word += wstride) {
    const int64_t k = k0 + word * kWave + l;
    int64_t b = 0, e = 0;
    if (k < k1) {
      b = newoff[k];
      e = newoff[k + 1];
    }
    const uint64_t hi = (uint64_t)(k - k0) << bc;
    const bool big = (e - b) > kLaneRow;
    if (!big)
      for (int64_t j = b; j < e; ++j) keys[j - base] = hi | (uint32_t)newcols[j];
    uint64_t hubs = ballot(big);
    while (hubs) {
      const int h = ffs64(hubs);
      hubs &= hubs - 1;
      const int64_t hb = shfl(b, h), he = shfl(e, h);
      const uint64_t hh = shfl(hi, h);
      for (int64_t j = hb + l; j < he; j += kWave) keys[j - base] = hh | (uint32_t)newcols[j];
    }
  }
}

// Relabel in batches of about kRelabelBatch entries once the graph has more
// than kRelabelWholeMax (the whole-graph pair sort needs 16 bytes per entry).
constexpr int64_t kRelabelWholeMax = (int64_t)1 << 32;
constexpr int64_t kRelabelBatch = (int64_t)1 << 30;

// Device buffers owned for the duration of one pass.
struct Bufs {
  std::vector<void*> ptrs;
  ~Bufs() {
    for (void* p : ptrs) (void)rbfs::dev_free(p);
  }
  template <class T>
  hipError_t alloc(T** out, int64_t count) {
    void* p = nullptr;
    hipError_t e = rbfs::dev_malloc(&p, sizeof(T) * (size_t)(count > 0 ? count : 1));
    if (e != hipSuccess) return e;
    ptrs.push_back(p);
    *out = (T*)p;
    return hipSuccess;
  }
  void forget(void* p) {
    for (auto& q : ptrs)
      if (q == p) q = nullptr;
  }
  // frees p now (a buffer of this pass no longer needed)
  void release(void* p) {
    for (auto& q : ptrs)
      if (q == p && q) {
        (void)rbfs::dev_free(q);
        q = nullptr;
      }
  }
};

}  // namespace

#define RCM_CHECK(x)                                                            \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      set_error(std::string("rcm_reorder: ") + #x + ": " + hipGetErrorString(e_)); \
      return e_ == hipErrorOutOfMemory ? -3 : -4;                                \
    }                                                                           \
  } while (0)

// Staged relabel: the old columns move to host memory (freeing their device
// copy), the relabelled column array is allocated, and slices of old
// rows come back one at a time to be renamed and copied to their new rows
// (sorted by the caller).  On failure after the move the old columns are
// put back on the device.
static int stage_relabel(Graph* g, int64_t n, int64_t nnz, const int32_t* perm,
                         const int64_t* newoff, uint64_t* kbuf, int64_t kcap, Bufs& B,
                         int32_t** newcols_out, hipStream_t stream) {
  int32_t* newcols = nullptr;
  int rc = 0;
  // ordinary (pageable) host memory: the copies go through the runtime's
  // own staging buffers, and nothing of this size is pinned
  int32_t* hcols = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz + kColPad));
  if (!hcols) {
    set_error("rcm_reorder: no host memory for the staged relabel");
    return -3;
  }
  hipError_t e = hipStreamSynchronize(stream);
  auto fail = [&](const char* what, hipError_t err) {
    set_error(std::string("rcm_reorder (staged relabel): ") + what + ": " +
              hipGetErrorString(err));
    return err == hipErrorOutOfMemory ? -3 : -4;
  };
  if (e == hipSuccess)
    e = hipMemcpy(hcols, g->cols, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    free(hcols);
    return fail("copy to host", e);
  }
  (void)rbfs::dev_free(g->cols);
  g->cols = nullptr;
  e = B.alloc(&newcols, nnz + kColPad);
  // old rows in slices of at most the key buffer's size (it is free now)
  int32_t* st = (int32_t*)kbuf;
  const int64_t per = std::max<int64_t>(1, kcap);  // int32 entries in 8 * kcap bytes / 2
  const int64_t nb = ceil_div(nnz, per);
  int64_t *kb = nullptr, *eb = nullptr;
  std::vector<int64_t> hkb, heb;
  if (e == hipSuccess) e = B.alloc(&kb, nb + 1);
  if (e == hipSuccess) e = B.alloc(&eb, nb + 1);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(batch_bounds_kernel, dim3(grid_for(nb + 1)), dim3(kBlock), 0, stream,
                       g->off, n, per, nb, kb, eb);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hkb.resize(nb + 1);
    heb.resize(nb + 1);
    e = hipMemcpyAsync(hkb.data(), kb, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost,
                       stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(heb.data(), eb, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost,
                       stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  for (int64_t i = 0; e == hipSuccess && i < nb; ++i) {
    const int64_t v0 = hkb[i], v1 = hkb[i + 1], e0 = heb[i], m = heb[i + 1] - heb[i];
    if (v1 <= v0 || m <= 0) continue;
    if (m > 2 * kcap) {  // a slice larger than the buffer: a row longer than kcap
      set_error("rcm_reorder: staged relabel slice larger than its buffer");
      rc = -1;
      break;
    }
    e = hipMemcpy(st, hcols + e0, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice);
    if (e != hipSuccess) break;
    const int64_t nw = ceil_div(v1 - v0, kWave);
    hipLaunchKernelGGL(scatter_rows_kernel,
                       dim3((unsigned)std::min<int64_t>(ceil_div(nw, kWavesPerBlock), 1 << 18)),
                       dim3(kBlock), 0, stream, g->off, v0, v1, e0, st, perm, newoff, newcols);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(stream);  // st is reused
  }
  if (e != hipSuccess || rc) {
    // put the old columns back so that the graph stays usable
    if (newcols) B.release(newcols);
    int32_t* back = nullptr;
    if (rbfs::dev_malloc(&back, sizeof(int32_t) * (size_t)(nnz + kColPad), stream) ==
            hipSuccess &&
        hipMemcpy(back, hcols, sizeof(int32_t) * (size_t)(nnz + kColPad),
                  hipMemcpyHostToDevice) == hipSuccess)
      g->cols = back;
    free(hcols);
    return rc ? rc : fail("slices", e);
  }
  free(hcols);
  *newcols_out = newcols;
  return 0;
}

int rcm_reorder_impl(Graph* g, hipStream_t stream, float* ms_out, int64_t keep_req) {
  const int64_t n = g->n, nnz = g->nnz;
  hipEvent_t e0, e1;
  RCM_CHECK(hipEventCreate(&e0));
  RCM_CHECK(hipEventCreate(&e1));
  RCM_CHECK(hipEventRecord(e0, stream));
  Bufs B;
  int32_t *deg, *nz, *vplus, *rank, *ccp, *csize, *label, *nextfree, *front, *next, *segstart,
      *counts, *tmpdeg, *chunk_pos, *perm, *iperm, *newdeg, *newcols;
  int64_t *pos_nz, *cbase, *qe, *newoff;
  uint32_t* plabel;
  unsigned long long* d_max;
  int* d_status;
  uint64_t *keys, *keys2;
  RCM_CHECK(B.alloc(&deg, n));
  RCM_CHECK(B.alloc(&nz, n));
  RCM_CHECK(B.alloc(&pos_nz, n + 1));
  RCM_CHECK(B.alloc(&d_max, 1));
  RCM_CHECK(B.alloc(&d_status, 1));
  RCM_CHECK(B.alloc(&counts, 3));
  RCM_CHECK(hipMemsetAsync(d_max, 0, sizeof(unsigned long long), stream));
  RCM_CHECK(hipMemsetAsync(d_status, 0, sizeof(int), stream));
  hipLaunchKernelGGL(deg_kernel, dim3(grid_folding(n)), dim3(kBlock), 0, stream, g->off, n, deg, nz,
                     d_max);
  RCM_CHECK(hipGetLastError());
  RCM_CHECK(scan_exclusive_i32(nz, pos_nz, n, g->scratch, stream));
  int64_t nplus = 0;
  unsigned long long maxdeg = 0;
  RCM_CHECK(hipMemcpyAsync(&nplus, pos_nz + n, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
  RCM_CHECK(hipMemcpyAsync(&maxdeg, d_max, sizeof(maxdeg), hipMemcpyDeviceToHost, stream));
  RCM_CHECK(hipStreamSynchronize(stream));
  // vertices of the Cuthill-McKee sequence that are reordered (all of V+
  // unless a partial order is asked for)
  const int64_t keep = (keep_req < 0 || keep_req > nplus) ? nplus : keep_req;
  const bool partial = keep < nplus;

  // 1. V+ ranked by (degree, id)
  const int bv = bits_for(n);
  const int bdeg = bits_for((int64_t)maxdeg + 1);
  // the relabel sorts the whole graph's pairs at once, or new rows in
  // batches of about `batch` entries when that would not fit (or when the
  // graph asks for batches)
  const int64_t batch = g->rcm_batch > 0 ? g->rcm_batch
                        : (nnz > kRelabelWholeMax ? kRelabelBatch : 0);
  const int64_t kcap = std::max<int64_t>(
      nplus, batch > 0 ? std::min<int64_t>(nnz, batch + (int64_t)maxdeg) : nnz);
  RCM_CHECK(B.alloc(&keys, kcap));
  RCM_CHECK(B.alloc(&keys2, kcap));
  RCM_CHECK(B.alloc(&vplus, nplus));
  RCM_CHECK(B.alloc(&rank, n));
  RCM_CHECK(B.alloc(&ccp, nplus));
  hipLaunchKernelGGL(deg_keys_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, deg, pos_nz, n,
                     bv, keys);
  RCM_CHECK(hipGetLastError());
  {
    uint64_t* k1 = keys;
    uint64_t* k2 = keys2;
    RCM_CHECK(radix_sort_u64(&k1, &k2, nplus, 0, bv + bdeg, g->scratch, stream));
    hipLaunchKernelGGL(vplus_kernel, dim3(grid_for(nplus)), dim3(kBlock), 0, stream, k1, nplus,
                       bv, vplus, rank, ccp);
    RCM_CHECK(hipGetLastError());
  }

  // 2. components (root = minimum rank) and 3. label bases
  const int64_t nwords = ceil_div(n, kWave);
  const int wgrid = (int)(ceil_div(nwords, kWavesPerBlock) < (1 << 18)
                              ? ceil_div(nwords, kWavesPerBlock) : (1 << 18));
  {
    int32_t* big_root = nullptr;
    RCM_CHECK(B.alloc(&big_root, 1));
    hipLaunchKernelGGL(cc_sample_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, g->off,
                       g->cols, n, rank, ccp);
    RCM_CHECK(hipGetLastError());
    if (nplus > 0) {
      // the last rank is a vertex of maximum degree: in the giant component
      // of the graphs this is built for (any choice is correct)
      hipLaunchKernelGGL(cc_big_root_kernel, dim3(1), dim3(1), 0, stream, ccp,
                         (int32_t)(nplus - 1), big_root);
      RCM_CHECK(hipGetLastError());
    } else {
      RCM_CHECK(hipMemsetAsync(big_root, 0xFF, sizeof(int32_t), stream));
    }
    hipLaunchKernelGGL(cc_union_kernel, dim3(wgrid), dim3(kBlock), 0, stream, g->off, g->cols, n,
                       rank, ccp, big_root);
    RCM_CHECK(hipGetLastError());
  }
  RCM_CHECK(B.alloc(&csize, nplus));
  RCM_CHECK(B.alloc(&cbase, nplus + 1));
  RCM_CHECK(hipMemsetAsync(csize, 0, sizeof(int32_t) * (nplus > 0 ? nplus : 1), stream));
  hipLaunchKernelGGL(cc_compress_kernel, dim3(grid_folding(nplus)), dim3(kBlock), 0, stream, ccp,
                     nplus, csize);
  RCM_CHECK(hipGetLastError());
  RCM_CHECK(scan_exclusive_i32(csize, cbase, nplus, g->scratch, stream));
  // component intervals of the final labelling, for searches to sweep only
  // the root's component
  int32_t* cflag = nullptr;
  int64_t* cpos = nullptr;
  int32_t* bounds = nullptr;
  int64_t ncomp = 0;
  RCM_CHECK(B.alloc(&cflag, nplus));
  RCM_CHECK(B.alloc(&cpos, nplus + 1));
  hipLaunchKernelGGL(comp_flag_kernel, dim3(grid_for(nplus)), dim3(kBlock), 0, stream, ccp, nplus,
                     cflag);
  RCM_CHECK(hipGetLastError());
  RCM_CHECK(scan_exclusive_i32(cflag, cpos, nplus, g->scratch, stream));
  RCM_CHECK(hipMemcpyAsync(&ncomp, cpos + nplus, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
  RCM_CHECK(hipStreamSynchronize(stream));
  RCM_CHECK(B.alloc(&bounds, ncomp + 1));
  hipLaunchKernelGGL(comp_bounds_kernel, dim3(grid_for(nplus)), dim3(kBlock), 0, stream, ccp,
                     cbase, cpos, nplus, ncomp, bounds);
  RCM_CHECK(hipGetLastError());

  // 4. level-synchronous Cuthill-McKee over all components
  uint64_t* lbits = nullptr;  // labelled vertices, one bit each
  RCM_CHECK(B.alloc(&label, n));
  RCM_CHECK(B.alloc(&lbits, ceil_div(n, kWave)));
  RCM_CHECK(B.alloc(&plabel, n));
  RCM_CHECK(B.alloc(&nextfree, nplus));
  RCM_CHECK(B.alloc(&front, nplus));
  RCM_CHECK(B.alloc(&next, nplus));
  RCM_CHECK(B.alloc(&segstart, nplus));
  RCM_CHECK(B.alloc(&tmpdeg, nplus));
  RCM_CHECK(B.alloc(&qe, nplus + 1));
  const int64_t chunk_cap = ceil_div(nnz, kChunkEdges) + 2;
  RCM_CHECK(B.alloc(&chunk_pos, chunk_cap));
  RCM_CHECK(hipMemsetAsync(label, 0xFF, sizeof(int32_t) * (size_t)n, stream));
  RCM_CHECK(hipMemsetAsync(plabel, 0xFF, sizeof(uint32_t) * (size_t)n, stream));
  RCM_CHECK(hipMemsetAsync(lbits, 0, sizeof(uint64_t) * (size_t)ceil_div(n, kWave), stream));
  RCM_CHECK(hipMemsetAsync(counts, 0, sizeof(int32_t) * 3, stream));
  hipLaunchKernelGGL(cm_roots_kernel, dim3(grid_for(nplus)), dim3(kBlock), 0, stream, ccp, cbase,
                     vplus, nplus, keep, label, lbits, nextfree, front, counts);
  RCM_CHECK(hipGetLastError());
  int32_t nf = 0;
  RCM_CHECK(hipMemcpyAsync(&nf, counts, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  RCM_CHECK(hipStreamSynchronize(stream));
  const int br = bits_for(nplus);
  int64_t labelled = nf;
  int status = 0;
  while (nf > 0) {
    hipLaunchKernelGGL(gather_deg_kernel, dim3(grid_for(nf)), dim3(kBlock), 0, stream, front,
                       (int64_t)nf, deg, tmpdeg);
    RCM_CHECK(hipGetLastError());
    RCM_CHECK(scan_exclusive_i32(tmpdeg, qe, nf, g->scratch, stream));
    hipLaunchKernelGGL(mark_kernel, dim3(grid_for(nf)), dim3(kBlock), 0, stream, qe, (int64_t)nf,
                       chunk_pos, chunk_cap);
    RCM_CHECK(hipGetLastError());
    int64_t E = 0;
    RCM_CHECK(hipMemcpyAsync(&E, qe + nf, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    RCM_CHECK(hipMemsetAsync(counts + 1, 0, sizeof(int32_t), stream));
    RCM_CHECK(hipStreamSynchronize(stream));
    const int64_t nchunks = ceil_div(E, kChunkEdges);
    if (nchunks > 0) {
      const int64_t gx = nchunks < 65536 ? nchunks : 65536;
      hipLaunchKernelGGL(cm_expand_kernel, dim3((unsigned)gx), dim3(kBlock), 0, stream, front, qe,
                         (int64_t)nf, E, chunk_pos, nchunks, g->off, g->cols, label, lbits, plabel,
                         next, counts + 1, nplus, d_status);
      RCM_CHECK(hipGetLastError());
    }
    int32_t m = 0;
    RCM_CHECK(hipMemcpyAsync(&m, counts + 1, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    RCM_CHECK(hipMemsetAsync(counts + 2, 0, sizeof(int32_t), stream));
    RCM_CHECK(hipMemcpyAsync(&status, d_status, sizeof(int), hipMemcpyDeviceToHost, stream));
    RCM_CHECK(hipStreamSynchronize(stream));
    if (status != 0 || m < 0 || m > nplus - labelled) {
      set_error("rcm_reorder: inconsistent level expansion (corrupt or non-canonical CSR?)");
      return -1;
    }
    if (m > 0) {
      hipLaunchKernelGGL(cm_keys_kernel, dim3(grid_for(m)), dim3(kBlock), 0, stream, next,
                         (int64_t)m, plabel, rank, br, keys);
      RCM_CHECK(hipGetLastError());
      uint64_t* k1 = keys;
      uint64_t* k2 = keys2;
      RCM_CHECK(radix_sort_u64(&k1, &k2, m, 0, 2 * br, g->scratch, stream));
      hipLaunchKernelGGL(cm_heads_kernel, dim3(grid_for(m)), dim3(kBlock), 0, stream, k1,
                         (int64_t)m, br, ccp, segstart);
      RCM_CHECK(hipGetLastError());
      hipLaunchKernelGGL(cm_assign_kernel, dim3(grid_folding(m)), dim3(kBlock), 0, stream, k1,
                         (int64_t)m, br, ccp, vplus, segstart, nextfree, keep, label, lbits,
                         front, counts + 2);
      RCM_CHECK(hipGetLastError());
      hipLaunchKernelGGL(cm_advance_kernel, dim3(grid_for(m)), dim3(kBlock), 0, stream, k1,
                         (int64_t)m, br, ccp, segstart, nextfree);
      RCM_CHECK(hipGetLastError());
    }
    // the next level expands the prefix labelled below keep (all of it in
    // a full pass)
    int32_t below = 0;
    if (m > 0) {
      RCM_CHECK(hipMemcpyAsync(&below, counts + 2, sizeof(int32_t), hipMemcpyDeviceToHost,
                               stream));
      RCM_CHECK(hipStreamSynchronize(stream));
    }
    if (below < 0 || below > m || (!partial && below != m)) {
      set_error("rcm_reorder: inconsistent level labels (corrupt or non-canonical CSR?)");
      return -1;
    }
    labelled += m;
    nf = below;
  }
  RCM_CHECK(hipMemcpyAsync(&status, d_status, sizeof(int), hipMemcpyDeviceToHost, stream));
  RCM_CHECK(hipStreamSynchronize(stream));
  if (status != 0 || labelled > nplus || (!partial && labelled != nplus)) {
    set_error("rcm_reorder: inconsistent labelling (corrupt or non-canonical CSR?)");
    return -1;
  }

  // 5. reversal, isolated vertices, relabelled CSR
  RCM_CHECK(B.alloc(&perm, n));
  RCM_CHECK(B.alloc(&iperm, n));
  int64_t* pos_rest = nullptr;
  if (partial) {
    // the rest of V+ keeps its id order: exclusive count of rest vertices
    int32_t* rflag = nullptr;
    RCM_CHECK(B.alloc(&rflag, n));
    RCM_CHECK(B.alloc(&pos_rest, n + 1));
    hipLaunchKernelGGL(rest_flag_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, deg, label,
                       n, keep, rflag);
    RCM_CHECK(hipGetLastError());
    RCM_CHECK(scan_exclusive_i32(rflag, pos_rest, n, g->scratch, stream));
    int64_t nrest = 0;
    RCM_CHECK(hipMemcpyAsync(&nrest, pos_rest + n, sizeof(int64_t), hipMemcpyDeviceToHost,
                             stream));
    RCM_CHECK(hipStreamSynchronize(stream));
    if (nrest != nplus - keep) {
      set_error("rcm_reorder: inconsistent partial labelling (corrupt or non-canonical CSR?)");
      return -1;
    }
  }
  hipLaunchKernelGGL(perm_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, deg, label, pos_nz,
                     pos_rest, n, nplus, keep, perm, iperm, d_status);
  RCM_CHECK(hipGetLastError());
  RCM_CHECK(B.alloc(&newdeg, n));
  RCM_CHECK(B.alloc(&newoff, n + 1));
  hipLaunchKernelGGL(newdeg_kernel, dim3(grid_for(n)), dim3(kBlock), 0, stream, iperm, deg, n,
                     newdeg);
  RCM_CHECK(hipGetLastError());
  RCM_CHECK(scan_exclusive_i32(newdeg, newoff, n, g->scratch, stream));
  // free what is no longer needed before the big sort
  RCM_CHECK(hipStreamSynchronize(stream));
  for (void* q : {(void*)deg, (void*)nz, (void*)pos_nz, (void*)vplus, (void*)rank, (void*)ccp,
                  (void*)csize, (void*)cbase, (void*)cflag, (void*)cpos, (void*)label,
                  (void*)lbits, (void*)plabel, (void*)nextfree, (void*)front, (void*)next,
                  (void*)segstart, (void*)tmpdeg, (void*)qe, (void*)chunk_pos, (void*)newdeg,
                  (void*)pos_rest})
    B.release(q);
  const int bn = bits_for(n);
  // the relabelled columns need nnz more entries next to the old ones; when
  // the device cannot hold both (the largest graphs), the old columns wait in
  // pinned host memory and come back a slice of old rows at a time
  bool staged = false;
  if (batch > 0) {
    size_t fr = 0, tot = 0;
    RCM_CHECK(hipMemGetInfo(&fr, &tot));
    const size_t need = sizeof(int32_t) * (size_t)(nnz + kColPad) + ((size_t)4 << 30);
    staged = g->rcm_stage > 0 || (g->rcm_stage == 0 && fr < need);
  }
  if (!staged) {
    RCM_CHECK(B.alloc(&newcols, nnz + kColPad));  // slack for aligned group reads
  }
  if (batch == 0) {
    hipLaunchKernelGGL(relabel_keys_kernel, dim3(wgrid), dim3(kBlock), 0, stream, g->off,
                       g->cols, n, nnz, perm, newoff, keys, d_status);
    RCM_CHECK(hipGetLastError());
    uint64_t* k1 = keys;
    uint64_t* k2 = keys2;
    RCM_CHECK(radix_sort_u64(&k1, &k2, nnz, 32, 32 + bn, g->scratch, stream));
    hipLaunchKernelGGL(groups_to_rows_kernel, dim3(wgrid), dim3(kBlock), 0, stream, g->off, n,
                       nnz, perm, newoff, k1, newcols, d_status);
    RCM_CHECK(hipGetLastError());
  } else {
    if (staged) {
      int rc = stage_relabel(g, n, nnz, perm, newoff, keys, kcap, B, &newcols, stream);
      if (rc) return rc;
    }
    // batches of new rows: keys ((k - k0) << bn | new column), sorted, back
    // into the rows
    const int64_t nb = ceil_div(nnz, batch);
    int64_t *kb = nullptr, *eb = nullptr;
    RCM_CHECK(B.alloc(&kb, nb + 1));
    RCM_CHECK(B.alloc(&eb, nb + 1));
    hipLaunchKernelGGL(batch_bounds_kernel, dim3(grid_for(nb + 1)), dim3(kBlock), 0, stream,
                       newoff, n, batch, nb, kb, eb);
    RCM_CHECK(hipGetLastError());
    std::vector<int64_t> hkb(nb + 1), heb(nb + 1);
    RCM_CHECK(hipMemcpyAsync(hkb.data(), kb, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost,
                             stream));
    RCM_CHECK(hipMemcpyAsync(heb.data(), eb, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost,
                             stream));
    RCM_CHECK(hipStreamSynchronize(stream));
    for (int64_t i = 0; i < nb; ++i) {
      const int64_t k0 = hkb[i], k1r = hkb[i + 1], m = heb[i + 1] - heb[i];
      if (k1r <= k0 || m <= 0) continue;
      if (m > kcap) {
        set_error("rcm_reorder: relabel batch larger than its buffer");
        return -1;
      }
      const int64_t nw = ceil_div(k1r - k0, kWave);
      const int rgrid = (int)std::min<int64_t>(ceil_div(nw, kWavesPerBlock), 1 << 18);
      if (staged)
        hipLaunchKernelGGL(inplace_keys_kernel, dim3(rgrid), dim3(kBlock), 0, stream, newoff, k0,
                           k1r, bn, newcols, keys);
      else
        hipLaunchKernelGGL(row_keys_kernel, dim3(rgrid), dim3(kBlock), 0, stream, g->off,
                           g->cols, iperm, perm, newoff, k0, k1r, bn, keys, kcap, d_status);
      RCM_CHECK(hipGetLastError());
      uint64_t* k1 = keys;
      uint64_t* k2 = keys2;
      RCM_CHECK(radix_sort_u64(&k1, &k2, m, 0, bn + bits_for(k1r - k0), g->scratch, stream));
      hipLaunchKernelGGL(keys_to_cols_kernel, dim3(grid_for(m)), dim3(kBlock), 0, stream, k1, m,
                         bn, newcols + heb[i]);
      RCM_CHECK(hipGetLastError());
    }
  }
  RCM_CHECK(hipMemcpyAsync(&status, d_status, sizeof(int), hipMemcpyDeviceToHost, stream));
  RCM_CHECK(hipEventRecord(e1, stream));
  RCM_CHECK(hipStreamSynchronize(stream));
  if (status != 0) {
    set_error("rcm_reorder: inconsistent labelling (corrupt or non-canonical CSR?)");
    return -1;
  }
  float ms = 0.f;
  RCM_CHECK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ms_out) *ms_out = ms;

  // install: the handle takes ownership of the new CSR and the permutation
  (void)rbfs::dev_free(g->off);
  if (g->cols) (void)rbfs::dev_free(g->cols);
  g->off = newoff;
  g->cols = newcols;
  g->perm = perm;
  g->iperm = iperm;
  // a partial order does not keep components in label intervals: searches
  // then sweep all of V+
  g->comp_bounds = partial ? nullptr : bounds;
  g->n_comp = partial ? 0 : ncomp;
  B.forget(newoff);
  B.forget(newcols);
  B.forget(perm);
  B.forget(iperm);
  if (!partial) B.forget(bounds);
  g->n_plus = nplus;
  g->n_sweep = nplus;
  g->reordered = 1;
  g->rcm_keep = keep;
  g->bytes += sizeof(int32_t) * 2 * (size_t)n + (partial ? 0 : sizeof(int32_t) * (size_t)(ncomp + 1));
  free_bfs_work(g);
  free_ms_work(g);
  g->scratch.release();
  return 0;
}

}  // namespace rbfs
