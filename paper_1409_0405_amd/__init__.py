"""MI355X-native flux reconstruction right-hand side (Euler / Navier-Stokes on
mixed prism/tet grids).  Importing the package loads nothing; the HIP library
binding lives in ``paper_1409_0405_amd.frlib`` and the seeded input
generators in ``paper_1409_0405_amd.inputs``."""
