// ntt_inst_c.hip - transform kernels for compute limb counts 15..22.
#include "ntt_impl.hpp"

namespace moma {

MOMA_NTT_INSTANTIATE(15) MOMA_NTT_INSTANTIATE(16) MOMA_NTT_INSTANTIATE(17) MOMA_NTT_INSTANTIATE(18) MOMA_NTT_INSTANTIATE(19) MOMA_NTT_INSTANTIATE(20) MOMA_NTT_INSTANTIATE(21) MOMA_NTT_INSTANTIATE(22)

}  // namespace moma
