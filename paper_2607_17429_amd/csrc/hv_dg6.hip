// H.V kernel instantiations for irrep dimension bucket 6.
#include "hv_kernel.h"

namespace ftlm {
namespace hvk {
FTLM_HV_INSTANTIATE(6)
}  // namespace hvk
}  // namespace ftlm
