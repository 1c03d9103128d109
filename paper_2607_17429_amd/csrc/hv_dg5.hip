// H.V kernel instantiations for irrep dimension bucket 5.
#include "hv_kernel.h"

namespace ftlm {
namespace hvk {
FTLM_HV_INSTANTIATE(5)
}  // namespace hvk
}  // namespace ftlm
