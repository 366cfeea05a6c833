// Batched EM-ADMM kernels with a fixed penalty over a box, one per shape class.
#include "batch_kernel.hpp"

namespace emx {

const ClassKernel *batch_class_table_admm() { return class_table_for<0, 0>(); }

}  // namespace emx
