// H.V kernel instantiations for irrep dimension bucket 3.
#include "hv_kernel.h"

namespace ftlm {
namespace hvk {
FTLM_HV_INSTANTIATE(3)
}  // namespace hvk
}  // namespace ftlm
