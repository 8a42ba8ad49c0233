// Instantiations of the derivative kernel (kept in their own translation
// unit so the library build compiles them in parallel).
#include "me_vjp_kernel.h"

namespace mf {

template hipError_t launch_vjp_one<GG_TT, double>(const VjpJob&, hipStream_t);
template hipError_t launch_vjp_one<GG_TT, float>(const VjpJob&, hipStream_t);
template hipError_t launch_vjp_one<GG_TTG, double>(const VjpJob&, hipStream_t);
template hipError_t launch_vjp_one<GG_TTG, float>(const VjpJob&, hipStream_t);

}  // namespace mf
