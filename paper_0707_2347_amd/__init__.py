"""Exact Strassen-Winograd products over Z/pZ on MI355X.

``capi`` binds the C-ABI of libwsmul.so (include/wsmul.h) one to one;
``api.mod_p_matmul`` is the same call on torch cuda tensors.
"""
