"""trimap: triangular-domain GPU kernels driven by the block-space map
lambda(omega) (Navarro, Bustos, Hitschfeld, arXiv 1609.01490), hand-written
HIP for AMD Instinct MI355X (gfx950) behind a C ABI (include/trimap.h).

Submodules: ``trimap`` (ctypes binding of ``libtrimap.so``; raises on import
if the library is not built), ``inputs`` (seeded synthetic inputs), ``build``
(hipcc build of the library: ``python -m paper_1609_01490_amd.build``).
"""
