"""MI355X (gfx950) executor for the UPIR data-parallel pattern.

The product is ``lib/libupir.so`` (C ABI in ``include/upir.h``); ``upir``
is its ctypes binding and ``helpers`` builds descriptors. Importing this
package does not load the library; ``upir.lib()`` does, and fails loudly
when it has not been built.
"""
from . import upir  # noqa: F401
