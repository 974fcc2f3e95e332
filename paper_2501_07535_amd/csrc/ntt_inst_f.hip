// ntt_inst_f.hip - transform kernels for compute limb counts 7..8.
#include "ntt_impl.hpp"

namespace moma {

MOMA_NTT_INSTANTIATE(7) MOMA_NTT_INSTANTIATE(8)

}  // namespace moma
