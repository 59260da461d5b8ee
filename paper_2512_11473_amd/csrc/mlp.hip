// Surrogate network for the near-surface integrals (filled in by the MLP
// kernels); until a model is created every call uses the plain integral.
#include "common.hpp"

namespace sgrid {

sgrid_status integrals_learned(const sgrid_grid *, const float *, const sgrid_mlp *, float *, uint32_t *,
                               hipStream_t) {
    set_error("no surrogate model support in this build");
    return SGRID_E_STATE;
}

}  // namespace sgrid
