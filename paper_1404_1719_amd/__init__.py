"""MI355X-native neutrino-matter interaction rates (energy-coupled kernels, l = 0, 1).

Importing the package loads nothing native; ``paper_1404_1719_amd.vtx`` binds the HIP
library and raises if it is missing."""
