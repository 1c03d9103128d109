// Fused small-block Lanczos kernel instantiations for irrep dimension bucket 1.
#include "lanczos_wg.h"

namespace ftlm {
namespace hvk {
FTLM_WG_INSTANTIATE(1)
}  // namespace hvk
}  // namespace ftlm
