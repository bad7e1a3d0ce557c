// pond_kernels25.hip -- the D2Q25 instantiation of the lattice-dependent
// kernels of the PonD f+g step (pond_lattice_kernels.h): D1Q5 x D1Q5 velocities
// (Table I), Grad order four, total or non-translational energy split.
#include "pond_lattice_kernels.h"

namespace pond {

template struct Launch<float, D2Q25>;
template struct Launch<double, D2Q25>;

}  // namespace pond
