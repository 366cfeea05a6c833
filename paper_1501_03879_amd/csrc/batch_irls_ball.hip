// Batched IRLS kernels for the smooth surrogate over a Euclidean ball, one per shape class.
#include "batch_kernel.hpp"

namespace emx {

const ClassKernel *batch_class_table_irls_ball() { return class_table_for<1, 1>(); }

}  // namespace emx
