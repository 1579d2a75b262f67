"""Differentiable SVD via polar decomposition on MI355X (gfx950).

The computation lives in ``libsvdp.so`` (C ABI in ``include/svdp.h``);
``api`` marshals torch tensors to it and ``autograd`` wraps it as
``torch.autograd.Function``s.  Importing this package loads nothing; the
first call loads the library and raises if it has not been built.
"""

__all__ = ["api", "autograd", "inputs", "predictor"]


def svd(A, **opts):
    from .autograd import svd as _svd
    return _svd(A, **opts)


def polar(A, **opts):
    from .autograd import polar as _polar
    return _polar(A, **opts)
