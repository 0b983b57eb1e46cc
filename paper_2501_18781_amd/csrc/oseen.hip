// oseen.hip -- matrix-free Q2 linearized momentum (Oseen) operator.
#include "kernels.hpp"

namespace mf {

hipError_t oseen_apply(const KMesh &, const OseenArgs &, int, const double *, double *, hipStream_t, const KTiming *)
{
    return hipErrorNotSupported;
}
hipError_t oseen_block_diagonal(const KMesh &, const OseenArgs &, double *, hipStream_t) { return hipErrorNotSupported; }

} // namespace mf
