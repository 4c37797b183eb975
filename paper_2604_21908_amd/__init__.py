"""MI355X-native MPO bond update for the middle-MPO contraction of mirrored
peaked circuits.  Importing the package loads nothing native; the HIP library
is loaded by :mod:`paper_2604_21908_amd.mpo` on first use."""
__all__ = ["circuitgen"]
