"""MI355X-native outer-product ("matrixized") stencil sweeps.

Importing the package is cheap: the HIP library is loaded on first use by
``paper_2310_16298_amd.stencil`` (see ``Plan``).
"""
__version__ = "0.1.0"
