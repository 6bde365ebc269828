"""MI355X (gfx950) RBF-FD hot path: stencil search, batched PHS + polynomial
weights, ghost closure and the fused right-hand side inside Runge-Kutta
stages, as hand-written HIP kernels behind the C ABI of include/rbffd.h.

Modules: ``rbffd`` (the binding; importing it raises ImportError when
librbffd.so is not built), ``pipeline`` (the ABI calls chained for the
paper's workloads) and ``build`` (hipcc build of the library).
"""
