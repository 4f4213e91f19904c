// inst_p2.hip -- kernel instantiations of precision path 2 (see node.hpp).
#include "fused.hpp"
#include "ops.hpp"

namespace mclbm {
const Ops *ops_prec2(int lattice, int model, bool rep) { return ops_for_lattice<2>(lattice, model, rep); }
}  // namespace mclbm
