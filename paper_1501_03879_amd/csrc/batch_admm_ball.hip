// Batched EM-ADMM kernels with a fixed penalty over a Euclidean ball, one per shape class.
#include "batch_kernel.hpp"

namespace emx {

const ClassKernel *batch_class_table_admm_ball() { return class_table_for<0, 1>(); }

}  // namespace emx
