// ntt_inst_g.hip - transform kernels for compute limb counts 28..32.
#include "ntt_impl.hpp"

namespace moma {

MOMA_NTT_INSTANTIATE(28) MOMA_NTT_INSTANTIATE(29) MOMA_NTT_INSTANTIATE(30) MOMA_NTT_INSTANTIATE(31) MOMA_NTT_INSTANTIATE(32)

}  // namespace moma
