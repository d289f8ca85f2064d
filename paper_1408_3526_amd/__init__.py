"""MI355X-native recursive multidimensional prediction-error filter.

The compute path is the HIP library ``librmdf.so`` (built from ``csrc/``);
``binding`` is a thin ctypes layer over its C ABI.  ``scenes`` draws seeded
synthetic inputs.  Importing this package loads nothing; ``binding.lib()``
loads the shared library and raises if it is missing.
"""
__all__ = ["binding", "scenes"]
