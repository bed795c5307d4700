"""MI355X-native constrained-least-squares radio image formation.

The compute path is the HIP library ``libclsimg.so`` (sources in ``csrc/``,
C ABI in ``include/clsimg.h``); ``clsimg`` is its Python binding.
"""

import os

PACKAGE_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PACKAGE_DIR, "libclsimg.so")
