// Reduced-precision contraction modes (split-BF16x3, FP8 with block scales).
#include "bqc_internal.h"

namespace bqc {

void launch_prepare_lowp(int precision, const DevInputs&, void*, Operands*, hipStream_t) {
    throw Error(-1, "precision " + std::to_string(precision) + " is not available in this build");
}

void launch_gemm_lowp(int precision, const GemmLaunch&, hipStream_t) {
    throw Error(-1, "precision " + std::to_string(precision) + " is not available in this build");
}

}  // namespace bqc
