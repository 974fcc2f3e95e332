// ntt_inst_a.hip - transform kernels for compute limb counts 1..8.
#include "ntt_impl.hpp"

namespace moma {

MOMA_NTT_INSTANTIATE(1) MOMA_NTT_INSTANTIATE(2) MOMA_NTT_INSTANTIATE(3) MOMA_NTT_INSTANTIATE(4) MOMA_NTT_INSTANTIATE(5) MOMA_NTT_INSTANTIATE(6) MOMA_NTT_INSTANTIATE(7) MOMA_NTT_INSTANTIATE(8)

}  // namespace moma
