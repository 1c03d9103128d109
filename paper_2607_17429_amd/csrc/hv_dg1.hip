// H.V kernel instantiations for irrep dimension bucket 1.
#include "hv_kernel.h"

namespace ftlm {
namespace hvk {
FTLM_HV_INSTANTIATE(1)
}  // namespace hvk
}  // namespace ftlm
