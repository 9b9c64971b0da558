"""MI355X (gfx950) solver for regularised Gaussian kernel systems (K_hat + gamma I) w = y.

Flexible GMRES preconditioned by inner CG solves of K_hat + delta I, with
on-the-fly kernel products in hand-written HIP (after Srinivasan et al.,
"Preconditioned Krylov solvers for kernel regression").

    from paper_1408_1237_amd import api
    w, info = api.fgmres_solve(x, sigma, gamma, y)

``api`` wraps the C ABI of ``libkrr.so`` (``include/krr.h``); ``native`` is the
raw ctypes binding; ``workloads`` draws the seeded synthetic inputs.
"""

__all__ = ["api", "native", "workloads", "autograd"]


def __getattr__(name):
    if name in __all__:
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
