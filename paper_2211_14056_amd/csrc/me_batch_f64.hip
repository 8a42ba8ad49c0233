// Instantiations of the persistent mixed-batch kernel (own translation unit
// so the build compiles them in parallel).
#include "me_batch_kernel.h"

namespace mf {

template hipError_t launch_batch_one<double, 0>(const BatchArgs&, int, int, hipStream_t);

}  // namespace mf
