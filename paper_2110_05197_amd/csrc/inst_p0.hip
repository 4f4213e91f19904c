// inst_p0.hip -- kernel instantiations of precision path 0 (see node.hpp).
#include "fused.hpp"
#include "ops.hpp"

namespace mclbm {
const Ops *ops_prec0(int lattice, int model, bool rep) { return ops_for_lattice<0>(lattice, model, rep); }
}  // namespace mclbm
