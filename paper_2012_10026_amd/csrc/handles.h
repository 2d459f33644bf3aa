// Definitions of the opaque handles of the C ABI.  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/rbfs.h"
#include "graph.h"

struct rbfs_graph {
  rbfs::Graph g;
};

struct rbfs_multi {
  rbfs::MsEngine eng;
  std::vector<rbfs::Graph*> gs;
  std::vector<int64_t> ubase;      // first union ID of each graph
  std::vector<int64_t> out_off;    // per-k output offset factor (sum of n before)
  int device = 0;
  // shape of the captured search
  int cap_k = 0, cap_mode = -1, cap_alpha = 0, cap_beta = 0;
  int32_t* cap_depth = nullptr;
  int32_t* cap_parent = nullptr;
  hipStream_t cap_stream = nullptr;
  hipStream_t own_stream = nullptr;  // used when the caller passes the NULL stream
};

