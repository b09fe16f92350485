"""Exact optimal cycle mean on AMD Instinct MI355X (gfx950).

Howard's policy iteration as data-parallel HIP kernels behind the C ABI of
``include/ocm.h``.  Submodules: ``ocm`` (the Python binding), ``synth``
(seeded input generators), ``build`` (hipcc build of ``libocm.so``).
"""
