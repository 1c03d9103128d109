// Fused small-block Lanczos kernel instantiations for irrep dimension bucket 8.
#include "lanczos_wg.h"

namespace ftlm {
namespace hvk {
FTLM_WG_INSTANTIATE(8)
}  // namespace hvk
}  // namespace ftlm
