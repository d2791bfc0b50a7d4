"""MI355X space-time Spline-Upwind isogeometric solver for the monodomain
equation with the Rogers-McCulloch ionic model.

The compute path is the HIP library ``libstiga.so`` (C ABI in
``include/st_iga.h``); ``binding`` marshals arguments to it.  Importing this
package does not load the library; ``binding.load()`` does, and raises if the
library has not been built.
"""
__all__ = ["binding", "build"]
