// Batched consensus ADMM with penalties mu w_k (weighted-mean z-update) over
// a Euclidean ball, one kernel per shape class.
#include "batch_kernel.hpp"

namespace emx {

const ClassKernel *batch_class_table_wpen_ball() { return class_table_for<4, 1>(); }

}  // namespace emx
