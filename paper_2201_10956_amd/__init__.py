"""epi3: exhaustive three-way epistasis scan (K2 score) for AMD MI355X (gfx950).

The compute path is the HIP library libepi3.so (C ABI in include/epi3.h);
`paper_2201_10956_amd.epi3` is its Python binding and raises ImportError when
the library has not been built (`paper_2201_10956_amd.build`).
"""
__all__ = ["epi3", "build"]
