"""MI355X-native real-time CC3 (arXiv 2407.18947): HIP kernels behind a C ABI.

`inputs` holds the seeded synthetic systems and field shapes; `_lib` is the
ctypes binding of librtcc3.so (include/rtcc3.h).  Importing the package loads
nothing; `_lib.load()` raises if the library has not been built.
"""
