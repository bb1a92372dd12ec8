"""MI355X (gfx950) library for compiled continuous-unitary-transformation graphs.

The compute path is libcutgraph.so (HIP kernels behind the C ABI declared in
include/cutgraph.h).  This package only marshals arguments:

* ``_lib``  -- ctypes binding, one function per C entry point, same names
* ``flow``  -- torch.autograd.Function running the RK4 coflow forward and its
               checkpointed discrete adjoint backward through the C ABI; and
               one for a single action with reverse (cut_graph_vjp) and
               forward-mode (cut_graph_jvp) derivatives

Importing raises if libcutgraph.so has not been built; nothing falls back to a
CPU implementation.
"""
from . import _lib  # noqa: F401  (fails loudly when the HIP library is missing)
from ._lib import *  # noqa: F401,F403
