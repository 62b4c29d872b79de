// Instantiations of the action kernels for the St Venant-Kirchhoff form.
#include "kernel_templates.h"

namespace femx {
Kernels lookup_svk(int dim, int degree, bool vjp)
{
    return lookup_form<FEM_SVK>(dim, degree, vjp);
}
}  // namespace femx
