"""ctypes binding placeholder (filled in with the C ABI)."""
__all__ = []
