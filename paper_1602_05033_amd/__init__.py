"""MI355X (gfx950) projection solver for symmetric Lyapunov and Sylvester
equations (Palitta & Simoncini, "Computationally enhanced projection methods
for symmetric Sylvester and Lyapunov matrix equations").

The solver itself is the HIP library ``liblyap.so`` behind the C ABI in
``include/lyap.h``; ``binding`` marshals PyTorch tensors into it.
"""
__all__ = ["binding", "build"]
