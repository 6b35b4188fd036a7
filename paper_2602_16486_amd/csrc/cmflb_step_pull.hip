// cmflb_step_pull.hip -- launches of the two-buffer pull step (every
// lattice, storage type and rate set), in a translation unit of their own.
#include "cmflb_step.h"

namespace cmf {

hipError_t launch_step_pull(int q, int storage, bool general, bool nt, const void *params,
                            const void *src, void *dst, const int64_t *step_ptr, int step_off,
                            double *partials, int grid, int block, hipStream_t stream) {
  return step_launch::by_lattice<false>(q, storage, general, nt, kStreamPull, params, src, dst,
                                        step_ptr, step_off, partials, grid, block, stream);
}

}  // namespace cmf
