// ntt_inst_b.hip - transform kernels for compute limb counts 9..12.
#include "ntt_impl.hpp"

namespace moma {

MOMA_NTT_INSTANTIATE(9) MOMA_NTT_INSTANTIATE(10) MOMA_NTT_INSTANTIATE(11) MOMA_NTT_INSTANTIATE(12)

}  // namespace moma
