// ntt_inst_d.hip - transform kernels for compute limb counts 5..6.
#include "ntt_impl.hpp"

namespace moma {

MOMA_NTT_INSTANTIATE(5) MOMA_NTT_INSTANTIATE(6)

}  // namespace moma
