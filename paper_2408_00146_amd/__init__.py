"""MI355X-native coupled central-moment lattice Boltzmann step (arXiv 2408.00146).

The GPU library is loaded lazily by :mod:`paper_2408_00146_amd.lbm`; importing
the package itself loads nothing.
"""
__all__ = ["cases", "lbm"]
