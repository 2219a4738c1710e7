// BF16 hi/lo split apply on matrix cores (batched path).
#include "safr_internal.h"

namespace safr {

hipError_t launch_cols_mfma(int, const MfmaArgs&, int, int, hipStream_t) { return hipErrorNotSupported; }

}  // namespace safr
