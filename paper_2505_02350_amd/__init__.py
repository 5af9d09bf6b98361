"""MI355X-native ERBF-fit hot path (SE-RBFNet optimisation step).

The computation lives in the HIP library ``liberbf.so`` behind the C ABI of
``include/erbf.h``; :mod:`.core` is its thin Python binding, :mod:`.autograd`
wraps evaluation and its vector-Jacobian product as a
``torch.autograd.Function``, and :mod:`.fit` drives optimisation steps
(captured in HIP graphs) for one or many shapes.
"""

__all__ = ["core", "build"]
