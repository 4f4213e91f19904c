// inst_p3.hip -- kernel instantiations of precision path 3 (see node.hpp).
#include "fused.hpp"
#include "ops.hpp"

namespace mclbm {
const Ops *ops_prec3(int lattice, int model, bool rep) { return ops_for_lattice<3>(lattice, model, rep); }
}  // namespace mclbm
