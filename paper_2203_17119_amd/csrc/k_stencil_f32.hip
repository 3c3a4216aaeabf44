// Stencil and s-local kernels instantiated for F32 storage (float arithmetic).
#include "k_stencil.inl"

namespace dwf {
int launch_stencil_f32(Context &c, const StencilSpec &sp, Field in, Field self, Field out)
{
    return launch_stencil_t<F32, float>(c, sp, in, self, out);
}
void launch_slocal_f32(Context &c, int op, Field in, Field out, int nbatch, long bstride)
{
    launch_slocal_t<F32, float>(c, op, in, out, nbatch, bstride);
}
}  // namespace dwf
