"""MI355X move stage of Gaussian-mixture SMC (arXiv 2503.16028).

`smc` is the binding of the C ABI in include/smc.h (libsmc.so, hand-written HIP for gfx950);
`sampler` drives the SMC loop of Alg. 1 through it; `build` compiles the library in-tree.
"""
