// H.V kernel instantiations for irrep dimension bucket 4.
#include "hv_kernel.h"

namespace ftlm {
namespace hvk {
FTLM_HV_INSTANTIATE(4)
}  // namespace hvk
}  // namespace ftlm
