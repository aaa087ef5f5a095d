"""Lazy, seed-consistent windowed diffusion sampling (InfiniteDiffusion) on
AMD Instinct MI355X: a C-ABI library of hand-written gfx950 HIP kernels
(include/td.h) and its Python binding (``paper_2512_08309_amd.td``)."""
