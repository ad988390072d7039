"""MI355X-native hot path of the matrix-free macro-element HDG method for
compressible Navier-Stokes (arXiv 2402.11361): a HIP C-ABI library
(libhdg.so) and a thin ctypes binding."""
