"""MI355X (gfx950) red-black Moebius domain-wall fermion solver library.

``paper_2203_17119_amd.dwf`` binds the C ABI of ``libdwf.so`` (include/dwf.h);
``paper_2203_17119_amd.synth`` draws the seeded synthetic inputs.  Importing
the package loads nothing; ``dwf.load()`` loads the HIP library and fails if
it has not been built.
"""
__all__ = ["dwf", "synth"]
