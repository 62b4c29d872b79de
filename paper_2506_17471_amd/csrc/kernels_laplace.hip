// Instantiations of the action kernels for the Laplace form.
#include "kernel_templates.h"

namespace femx {
Kernels lookup_laplace(int dim, int degree, bool vjp)
{
    return lookup_form<FEM_LAPLACE>(dim, degree, vjp);
}
}  // namespace femx
