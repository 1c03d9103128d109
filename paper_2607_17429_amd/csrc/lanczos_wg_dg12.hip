// Fused small-block Lanczos kernel instantiations for irrep dimension bucket 12.
#include "lanczos_wg.h"

namespace ftlm {
namespace hvk {
FTLM_WG_INSTANTIATE(12)
}  // namespace hvk
}  // namespace ftlm
