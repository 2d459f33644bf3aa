// Edge-balanced frontier expansion.
//
// A frontier is a list of vertices q[0..nq) with the exclusive prefix sum of
// their degrees qe[0..nq] (qe[nq] = E).  The E adjacency entries of the
// frontier, taken in list order, are cut into chunks of 2^cshift entries
// (at most kChunkEdges); chunk c starts at entry c << cshift, and
// chunk_pos[c] is the list position whose row holds that entry.  A
// workgroup stages the list positions a chunk touches in LDS and each thread
// finds the position of its entry by binary search there, so every thread
// handles the same number of entries whatever the degree skew, and
// consecutive threads read consecutive column entries.  This is the GPU counterpart of the paper's
// even split of each frontier vertex's neighbours over the threads (top-down
// load balancing, Algorithm 4 and Eq. 3).
#pragma once
#include "common.h"
#include "graph.h"

namespace rbfs {

// Marks the chunks whose first entry lies in [base, base + deg) as starting at
// list position pos.
__device__ __forceinline__ void mark_chunks(int32_t* chunk_pos, int64_t chunk_cap, int64_t base,
                                            int64_t deg, int32_t pos,
                                            int cshift = kChunkShift) {
  const int64_t cm = ((int64_t)1 << cshift) - 1;
  const int64_t c0 = (base + cm) >> cshift;
  const int64_t c1 = (base + deg + cm) >> cshift;
  for (int64_t c = c0; c < c1 && c < chunk_cap; ++c) chunk_pos[c] = pos;
}

struct ChunkLds {
  int64_t qe[kChunkEdges + 2];
  int64_t rowoff[kChunkEdges + 2];
  int32_t u[kChunkEdges + 2];
  int32_t k;
};

// Processes chunk c.  f(active, u, w) is called by every thread of the block
// in lock-step rounds of BLOCK entries (inactive threads get active = false),
// so f may use wave-wide operations.  Returns false if the chunk touched more
// list positions than fit in LDS (corrupt input).
template <int BLOCK, class F>
__device__ __forceinline__ bool expand_chunk(ChunkLds& s, int64_t c, int64_t E, const int32_t* q,
                                             const int64_t* qe, int64_t nq,
                                             const int32_t* chunk_pos, int64_t nchunks,
                                             const int64_t* off, const int32_t* cols, F&& f,
                                             int cshift = kChunkShift) {
  const int64_t ch = (int64_t)1 << cshift;
  const int64_t e0 = c << cshift;
  const int64_t e1 = (e0 + ch < E) ? e0 + ch : E;
  if (threadIdx.x == 0) {
    const int64_t p0 = chunk_pos[c];
    const int64_t p1 = (c + 1 < nchunks) ? (int64_t)chunk_pos[c + 1] : nq - 1;
    int64_t k = p1 - p0 + 1;
    const bool bad = p0 < 0 || p1 >= nq || k < 1 || k > kChunkEdges + 1 ||
                     cshift > kChunkShift;
    s.k = bad ? -1 : (int32_t)k;
    s.u[kChunkEdges + 1] = (int32_t)p0;
  }
  __syncthreads();
  const int32_t k = s.k;
  if (k < 0) return false;
  const int64_t p0 = s.u[kChunkEdges + 1];
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += BLOCK) {
    const int32_t u = q[p0 + i];
    s.qe[i] = qe[p0 + i];
    s.u[i] = u;
    s.rowoff[i] = off[u];
  }
  __syncthreads();
  for (int64_t base = e0; base < e1; base += BLOCK) {
    const int64_t e = base + threadIdx.x;
    const bool active = e < e1;
    int32_t u = 0, w = 0;
    if (active) {
      int lo = 0, hi = k - 1;  // last i with qe[i] <= e
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.qe[mid] <= e) lo = mid; else hi = mid - 1;
      }
      u = s.u[lo];
      w = cols[s.rowoff[lo] + (e - s.qe[lo])];
    }
    f(active, u, w);
  }
  __syncthreads();
  return true;
}

// Chunk staging for expand_chunk_batch: up to CAP entries per chunk.  Row
// starts are kept relative to the chunk start (the first one clamped to 0),
// with the column base of each row (row offset minus row start), so an
// entry's column index is colbase + entry.
template <int CAP>
struct ChunkLdsB {
  int64_t colbase[CAP + 2];
  int32_t qe[CAP + 2];
  int32_t u[CAP + 2];
  int32_t k;
  int32_t p0;
};

// expand_chunk with K entries per thread: entry r * BLOCK + threadIdx.x of
// each round of K * BLOCK entries goes to slot r, and f(act, u, w) receives
// the K slots at once, so it can issue the K entries' memory accesses
// together instead of one dependent chain at a time.  Chunks may hold up to
// K * BLOCK entries (cshift at most log2(K * BLOCK)).
template <int BLOCK, int K, class F>
__device__ __forceinline__ bool expand_chunk_batch(ChunkLdsB<K * BLOCK>& s, int64_t c, int64_t E,
                                                   const int32_t* q, const int64_t* qe,
                                                   int64_t nq, const int32_t* chunk_pos,
                                                   int64_t nchunks, const int64_t* off,
                                                   const int32_t* cols, int cshift, F&& f) {
  constexpr int CAP = K * BLOCK;
  const int64_t e0 = c << cshift;
  const int64_t e1 = (e0 + ((int64_t)1 << cshift) < E) ? e0 + ((int64_t)1 << cshift) : E;
  const int n = (int)(e1 - e0);
  if (threadIdx.x == 0) {
    const int64_t p0 = chunk_pos[c];
    const int64_t p1 = (c + 1 < nchunks) ? (int64_t)chunk_pos[c + 1] : nq - 1;
    const int64_t k = p1 - p0 + 1;
    const bool bad = p0 < 0 || p1 >= nq || k < 1 || k > CAP + 1 || ((int64_t)1 << cshift) > CAP;
    s.k = bad ? -1 : (int32_t)k;
    s.p0 = (int32_t)p0;
  }
  __syncthreads();
  const int32_t k = s.k;
  if (k < 0) return false;
  const int64_t p0 = s.p0;
  for (int i = threadIdx.x; i < k; i += BLOCK) {
    const int32_t u = q[p0 + i];
    const int64_t a = qe[p0 + i];
    s.u[i] = u;
    s.qe[i] = (int32_t)(a > e0 ? a - e0 : 0);
    s.colbase[i] = off[u] - a;
  }
  __syncthreads();
  for (int base = 0; base < n; base += CAP) {
    bool act[K];
    int32_t u[K], w[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
      const int e = base + r * BLOCK + (int)threadIdx.x;
      act[r] = e < n;
      int lo = 0, hi = k - 1;  // last i with qe[i] <= e
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.qe[mid] <= e) lo = mid; else hi = mid - 1;
      }
      u[r] = act[r] ? s.u[lo] : 0;
      w[r] = act[r] ? cols[s.colbase[lo] + e0 + e] : 0;
    }
    f(act, u, w);
  }
  __syncthreads();
  return true;
}

}  // namespace rbfs
