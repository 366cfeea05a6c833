// Batched EM-ADMM kernels with the adaptive penalty over a box, one per shape class.
#include "batch_kernel.hpp"

namespace emx {

const ClassKernel *batch_class_table_adapt() { return class_table_for<2, 0>(); }

}  // namespace emx
