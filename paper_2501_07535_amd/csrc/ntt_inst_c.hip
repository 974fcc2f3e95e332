// ntt_inst_c.hip - transform kernels for compute limb counts 15..16.
#include "ntt_impl.hpp"

namespace moma {

MOMA_NTT_INSTANTIATE(15) MOMA_NTT_INSTANTIATE(16)

}  // namespace moma
