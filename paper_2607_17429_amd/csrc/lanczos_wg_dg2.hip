// Fused small-block Lanczos kernel instantiations for irrep dimension bucket 2.
#include "lanczos_wg.h"

namespace ftlm {
namespace hvk {
FTLM_WG_INSTANTIATE(2)
}  // namespace hvk
}  // namespace ftlm
