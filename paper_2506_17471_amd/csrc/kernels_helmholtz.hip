// Instantiations of the action kernels for the Helmholtz form.
#include "kernel_templates.h"

namespace femx {
Kernels lookup_helmholtz(int dim, int degree, bool vjp)
{
    return lookup_form<FEM_HELMHOLTZ>(dim, degree, vjp);
}
}  // namespace femx
