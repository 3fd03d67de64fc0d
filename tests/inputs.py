"""The seeded input recipes, for the tests (they live in the package, beside
the benchmark and the run drivers that also start from them)."""
from paper_2201_10132_amd.inputs import *  # noqa: F401,F403
from paper_2201_10132_amd.inputs import _M64  # noqa: F401
