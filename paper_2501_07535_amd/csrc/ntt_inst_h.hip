// ntt_inst_h.hip - transform kernels for compute limb counts 13..14.
#include "ntt_impl.hpp"

namespace moma {

MOMA_NTT_INSTANTIATE(13) MOMA_NTT_INSTANTIATE(14)

}  // namespace moma
