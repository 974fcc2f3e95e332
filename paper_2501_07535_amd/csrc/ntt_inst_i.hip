// ntt_inst_i.hip - transform kernels for compute limb counts 17..22.
#include "ntt_impl.hpp"

namespace moma {

MOMA_NTT_INSTANTIATE(17) MOMA_NTT_INSTANTIATE(18) MOMA_NTT_INSTANTIATE(19) MOMA_NTT_INSTANTIATE(20) MOMA_NTT_INSTANTIATE(21) MOMA_NTT_INSTANTIATE(22)

}  // namespace moma
