"""Whittle-Matern Gaussian random fields on surfaces by isogeometric FEM on one AMD MI355X.

The computation lives in libgfield.so (HIP, gfx950) behind the C ABI of include/gfield.h;
`paper_2605_24882_amd.gfield` is its ctypes binding, `paper_2605_24882_amd.build` builds it,
`paper_2605_24882_amd.inputs` generates seeded synthetic inputs.
"""
