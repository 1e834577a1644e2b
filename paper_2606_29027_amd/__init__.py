"""MI355X (gfx950) implementation of the SLAR / LoMaC time step.

``lib`` is the ctypes binding of the HIP library ``libslar.so``
(built by ``build.build()``); ``solver`` drives one time step through it.
Importing the package loads nothing; the library is loaded on first use and
a missing library raises instead of falling back to any CPU path.
"""
__all__ = ["lib", "solver", "build"]
