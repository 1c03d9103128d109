// Fused small-block Lanczos kernel instantiations for irrep dimension bucket 6.
#include "lanczos_wg.h"

namespace ftlm {
namespace hvk {
FTLM_WG_INSTANTIATE(6)
}  // namespace hvk
}  // namespace ftlm
