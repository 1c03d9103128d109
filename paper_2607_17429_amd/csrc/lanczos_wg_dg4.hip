// Fused small-block Lanczos kernel instantiations for irrep dimension bucket 4.
#include "lanczos_wg.h"

namespace ftlm {
namespace hvk {
FTLM_WG_INSTANTIATE(4)
}  // namespace hvk
}  // namespace ftlm
