// Instantiations of the action kernels for the neo-Hookean form.
#include "kernel_templates.h"

namespace femx {
Kernels lookup_neohookean(int dim, int degree, bool vjp)
{
    return lookup_form<FEM_NEOHOOKEAN>(dim, degree, vjp);
}
}  // namespace femx
