// Instantiations of the action kernels for the elasticity form.
#include "kernel_templates.h"

namespace femx {
Kernels lookup_elasticity(int dim, int degree, bool vjp)
{
    return lookup_form<FEM_ELASTICITY>(dim, degree, vjp);
}
}  // namespace femx
