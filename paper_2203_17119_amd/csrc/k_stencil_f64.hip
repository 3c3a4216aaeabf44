// Stencil and s-local kernels instantiated for F64 storage (double arithmetic).
#include "k_stencil.inl"

namespace dwf {
int launch_stencil_f64(Context &c, const StencilSpec &sp, Field in, Field self, Field out)
{
    return launch_stencil_t<F64, double>(c, sp, in, self, out);
}
void launch_slocal_f64(Context &c, int op, Field in, Field out, int nbatch, long bstride)
{
    launch_slocal_t<F64, double>(c, op, in, out, nbatch, bstride);
}
}  // namespace dwf
