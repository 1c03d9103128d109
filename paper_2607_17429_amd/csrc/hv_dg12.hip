// H.V kernel instantiations for irrep dimension bucket 12.
#include "hv_kernel.h"

namespace ftlm {
namespace hvk {
FTLM_HV_INSTANTIATE(12)
}  // namespace hvk
}  // namespace ftlm
