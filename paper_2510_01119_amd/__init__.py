"""gs4d: an MI355X-native differentiable 4D Gaussian-splatting rasterizer.

Importing the package loads nothing; the HIP library is loaded on first use
by :mod:`paper_2510_01119_amd.gs4d`.
"""
__all__ = ["gs4d", "synth"]
