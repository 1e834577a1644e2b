// Learned preconditioner for the Krylov solve of the macroscopic system.
#include "slar_internal.h"
#include "lomac.h"

namespace slar {
hipError_t cnn_apply(hipStream_t s, Workspace* ws, const slar_cnn* net, const double* v,
                     const double* U, double* z) {
  (void)s; (void)ws; (void)net; (void)v; (void)U; (void)z;
  return hipErrorNotSupported;
}
}  // namespace slar
