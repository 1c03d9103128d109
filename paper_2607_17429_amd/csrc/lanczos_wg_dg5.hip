// Fused small-block Lanczos kernel instantiations for irrep dimension bucket 5.
#include "lanczos_wg.h"

namespace ftlm {
namespace hvk {
FTLM_WG_INSTANTIATE(5)
}  // namespace hvk
}  // namespace ftlm
