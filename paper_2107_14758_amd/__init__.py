"""MI355X-native vertex-star FDM/sparse relaxation solver for high-order FEM.

The compute path lives in the HIP/C++ shared library built from ``csrc/``
(C ABI declared in ``include/vsr.h``); ``vsr`` is its thin ctypes binding and
``inputs`` holds the seeded synthetic workload generators.  Importing this
package loads nothing; ``paper_2107_14758_amd.vsr`` loads the library.
"""
