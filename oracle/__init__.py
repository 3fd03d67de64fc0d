"""FP64 CPU oracle for the two-fluid kinetic scheme (arXiv:2201.10132).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_2201_10132_amd``) never imports, links or calls it, and the two share
no code.

The scheme's arithmetic lives in ``tpl_oracle.c`` (plain C, FP64); this module
only compiles it and marshals numpy arrays through ctypes.  ``learned.py``
holds the FP64 numpy reference of the learned coarse-lattice correction
(network, training update, restriction, features, momentum source).
"""
from .oracle import OracleSim, build, lib_path, max_threads, set_threads, splitmix64_next  # noqa: F401
