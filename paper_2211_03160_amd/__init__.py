"""MI355X-native thermal lattice Boltzmann step (DDF MRT, arXiv:2211.03160).

Importing the package loads nothing; ``paper_2211_03160_amd.lbm`` holds the
binding of the HIP library.
"""
