// cmflb_step_aa.hip -- launches of the in-place (AA) step pair (every
// lattice, storage type and rate set), in a translation unit of their own.
#include "cmflb_step.h"

namespace cmf {

hipError_t launch_step_in_place(int q, int storage, bool general, bool nt, bool odd,
                                const void *params, void *buf, const int64_t *step_ptr,
                                int step_off, double *partials, int grid, int block,
                                hipStream_t stream) {
  return step_launch::by_lattice<true>(q, storage, general, nt, odd ? kStreamAAOdd : kStreamAAEven,
                                       params, buf, buf, step_ptr, step_off, partials, grid, block,
                                       stream);
}

}  // namespace cmf
