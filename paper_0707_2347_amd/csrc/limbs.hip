// Base products from signed 8-bit digits of centred residues (INT8 matrix cores).
#include "wsmul_internal.hpp"

namespace wsmul {

bool limbs_supported(int64_t p) { return p <= 16711423; }

hipError_t launch_gemm_limbs(const ws_op_desc &op, const DevBufs &bufs, int dtype, int64_t p,
                             hipStream_t stream) {
    (void)op; (void)bufs; (void)dtype; (void)p; (void)stream;
    return hipErrorNotSupported;
}

}  // namespace wsmul
