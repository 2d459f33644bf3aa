// placeholder, replaced by the bit-parallel search
#include "graph.h"
#include "../../include/rbfs.h"
namespace rbfs {
void free_ms_work(Graph* g) { (void)g; }
int bfs_batch_impl(Graph*, const int32_t*, int32_t, int32_t*, int32_t*, int, int, int, int,
                   hipStream_t, void*) {
  set_error("bfs_batch: not built");
  return RBFS_E_UNSUPPORTED;
}
}  // namespace rbfs
