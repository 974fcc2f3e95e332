// ntt_inst_a.hip - transform kernels for compute limb counts 1..4.
#include "ntt_impl.hpp"

namespace moma {

MOMA_NTT_INSTANTIATE(1) MOMA_NTT_INSTANTIATE(2) MOMA_NTT_INSTANTIATE(3) MOMA_NTT_INSTANTIATE(4)

}  // namespace moma
