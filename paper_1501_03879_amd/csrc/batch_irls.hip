// Batched IRLS kernels for the smooth surrogate over a box, one per shape class.
#include "batch_kernel.hpp"

namespace emx {

const ClassKernel *batch_class_table_irls() { return class_table_for<1, 0>(); }

}  // namespace emx
