"""MI355X-native CSP solver (the CUBICS design of "Experimenting with
Constraint Programming on GPU", re-built for gfx950).

The solver is the HIP library ``libcubics.so`` behind the C ABI in
``include/cubics.h``; :mod:`paper_1909_09213_amd.cubics` is its Python
binding.  Importing the package does not load the library; the binding
raises ImportError if it has not been built.
"""

__all__ = ["cubics", "build"]
