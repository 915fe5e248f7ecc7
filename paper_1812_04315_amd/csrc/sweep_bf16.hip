// BF16 sweeps (precision form): X in bfloat16, FP32 accumulation on MFMA.
#include "internal.hpp"

namespace cnmf {

size_t sweep_right_bf16_partial_floats(const Dev&, int64_t, int64_t) { return 0; }
size_t sweep_left_bf16_partial_floats(const Dev&, int64_t, int64_t) { return 0; }

hipError_t sweep_right_bf16(const Dev&, int64_t, int64_t, const uint16_t*, int64_t, int,
                            const float*, int64_t, float*, int64_t, float*, uint16_t*) {
    return hipErrorNotSupported;
}
hipError_t sweep_left_bf16(const Dev&, int64_t, int64_t, const uint16_t*, int64_t, int,
                           const float*, int64_t, float*, int64_t, bool, float*, uint16_t*) {
    return hipErrorNotSupported;
}

}  // namespace cnmf
