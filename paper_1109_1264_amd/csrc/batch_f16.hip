// batch_f16.hip -- the batched kernels for one element type (compiled
// separately so the types build in parallel).
#include "batch_kernels.hpp"

namespace salt {
BatchFn batch_launcher_f16(int id) { return batch_launcher_for<SALT_F16>(id); }
BatchFn batch_multi_launcher_f16() { return &launch_batch_multi<SALT_F16>; }
BatchFn batch_combine_launcher_f16() { return &launch_combine<SALT_F16>; }
}  // namespace salt
