// kernels_f64.hip -- the parity instantiation: the same transport source in
// IEEE double precision, built without FMA contraction so that every step
// rounds as the FP64 CPU reference does.
#include "kernels_impl.hpp"

namespace omc {
template struct Launch<double>;
}  // namespace omc
