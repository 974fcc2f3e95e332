// ntt_inst_e.hip - transform kernels for compute limb counts 5..8.
#include "ntt_impl.hpp"

namespace moma {

MOMA_NTT_INSTANTIATE(5) MOMA_NTT_INSTANTIATE(6) MOMA_NTT_INSTANTIATE(7) MOMA_NTT_INSTANTIATE(8)

}  // namespace moma
