// H.V kernel instantiations for irrep dimension bucket 2.
#include "hv_kernel.h"

namespace ftlm {
namespace hvk {
FTLM_HV_INSTANTIATE(2)
}  // namespace hvk
}  // namespace ftlm
