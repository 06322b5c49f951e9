"""MI355X-native Wilson-Dirac operator, CG solvers and fermion force for SU(2).

Submodules:

* ``hrd``      — binding of the HIP library ``libhrd.so`` (loaded on import of
  that submodule, never by the package itself);
* ``autograd`` — ``torch.autograd.Function`` wrappers over the binding;
* ``inputs``   — seeded synthetic gauge and spinor fields (numpy only).
"""
