// H.V kernel instantiations for irrep dimension bucket 8.
#include "hv_kernel.h"

namespace ftlm {
namespace hvk {
FTLM_HV_INSTANTIATE(8)
}  // namespace hvk
}  // namespace ftlm
