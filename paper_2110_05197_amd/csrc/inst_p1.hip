// inst_p1.hip -- kernel instantiations of precision path 1 (see node.hpp).
#include "fused.hpp"
#include "ops.hpp"

namespace mclbm {
const Ops *ops_prec1(int lattice, int model, bool rep) { return ops_for_lattice<1>(lattice, model, rep); }
}  // namespace mclbm
