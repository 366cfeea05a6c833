// Batched consensus ADMM with penalties mu w_k (weighted-mean z-update) over
// a box, one kernel per shape class.
#include "batch_kernel.hpp"

namespace emx {

const ClassKernel *batch_class_table_wpen() { return class_table_for<4, 0>(); }

}  // namespace emx
