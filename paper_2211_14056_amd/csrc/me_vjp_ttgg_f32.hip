// Instantiations of the derivative kernel (kept in their own translation
// unit so the library build compiles them in parallel).
#include "me_vjp_kernel.h"

namespace mf {

template hipError_t launch_vjp_batch_one<GG_TTGG, float>(const VjpBatchArgs&, hipStream_t);

}  // namespace mf
