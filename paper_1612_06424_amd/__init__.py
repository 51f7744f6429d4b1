"""MI355X-native Wilson-Dirac hot path of the factorised quark propagator
(Ce, Giusti, Schaefer, arXiv:1612.06424).

The compute path is the HIP library ``libdd.so`` (C ABI, ``include/dd.h``);
``paper_1612_06424_amd.dd`` is its thin Python binding.  Importing the package
does not load the library; importing ``paper_1612_06424_amd.dd`` does, and
fails loudly when it has not been built.
"""
__all__ = ["dd", "inputs"]
