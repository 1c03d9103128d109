// Fused small-block Lanczos kernel instantiations for irrep dimension bucket 3.
#include "lanczos_wg.h"

namespace ftlm {
namespace hvk {
FTLM_WG_INSTANTIATE(3)
}  // namespace hvk
}  // namespace ftlm
