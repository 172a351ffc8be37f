"""MI355X-native exact temporal motif mining.

The mining runs in the HIP library ``libtmotif.so`` (C ABI in
``include/tmotif.h``); ``api`` is its Python binding and ``synth`` draws seeded
synthetic inputs. Importing this package does not load the library; the first
API call does, and fails loudly if it has not been built.
"""

__all__ = ["api", "synth"]
