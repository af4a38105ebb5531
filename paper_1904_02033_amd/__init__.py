"""MI355X homomorphic distance stage of secure approximate k-NN search.

``native`` is the ctypes binding of the C ABI in include/sanns.h (the HIP
library libsanns.so); ``stage`` wraps it for torch device tensors;
``topk`` reconstructs distances from shares and selects neighbours;
``serve`` is the continuous-batching request loop.
"""
__all__ = ["native", "stage"]
