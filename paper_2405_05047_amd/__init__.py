"""MI355X-native adaptive-Q1 geometric multigrid (HIP kernels behind a C ABI).

Submodules:
  gen   ctypes binding of the native problem generator (libmggen.so)
  mg    ctypes binding of the HIP solver library (libmgq1.so)
  build compiles both libraries in-tree
Importing the package loads nothing; the bindings load their library on first use and
raise if it is missing.
"""
