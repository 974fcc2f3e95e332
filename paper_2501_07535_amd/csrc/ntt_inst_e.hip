// ntt_inst_e.hip - transform kernels for compute limb counts 23..27.
#include "ntt_impl.hpp"

namespace moma {

MOMA_NTT_INSTANTIATE(23) MOMA_NTT_INSTANTIATE(24) MOMA_NTT_INSTANTIATE(25) MOMA_NTT_INSTANTIATE(26) MOMA_NTT_INSTANTIATE(27)

}  // namespace moma
