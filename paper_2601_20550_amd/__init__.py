"""MI355X-native HEOM-2DVS hot path: HIP kernels behind a C ABI plus a ctypes binding.

Importing the package loads libheom2dvs.so and fails loudly if it is missing.
PyTorch, when installed, is imported first so that the process uses the HIP
runtime torch ships with (both carry the soname libamdhip64.so.7).
"""

try:  # noqa: SIM105
    import torch  # noqa: F401
except ImportError:  # torch is optional plumbing (streams, allocator)
    pass

from .heom2dvs import *  # noqa: F401,F403,E402
from .heom2dvs import Model, State, load_library  # noqa: F401,E402

load_library()
