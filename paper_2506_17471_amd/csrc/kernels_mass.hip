// Instantiations of the action kernels for the mass form.
#include "kernel_templates.h"

namespace femx {
Kernels lookup_mass(int dim, int degree, bool vjp)
{
    return lookup_form<FEM_MASS>(dim, degree, vjp);
}
}  // namespace femx
