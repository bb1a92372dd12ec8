"""Plain FP64 CPU oracle for the compiled-CUT-graph hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, links or calls this package; only the test suite, the
smoke check and the benchmark's CPU-baseline leg do.  It shares no code with the
GPU path: it has its own registries, its own record generation, its own graph
actions, generators, integrator and adjoint.

Every function follows the paper (Peng & Govind, "Compile-once operation graphs
for reusable continuous unitary transformations") at the passage named in its
docstring:

* Sec. 2.1, Eqs. (coflow), (block-generator), (projected-flow): the projected CUT
  flow dH/ds = P[eta(H), H], dX/ds = P[eta(H), X].
* Sec. 2.2, Eq. (graph-actions): records (target k, left i, right j, factor c)
  grouped by target; an action is a sum over the target's records.
* Sec. 2.4, Eqs. (forward-coeff), (dual), (duality-invariant) and the graph-level
  adjoint paragraph: the adjoint accumulates the same factor into the input
  coordinate; Eq. (directional-derivative): the derivative of one action is the
  induced generator variation plus the linear response to the operand.

Modules:
  algebra   registries and contribution records, from the operator algebra
  graph     forward action, the two adjoint traversals
  gen       generators (Wegner graph pass; G2 normalised Wegner), their JVPs
            and VJPs
  deriv     directional derivative and transpose of one projected action
            (Eq. directional-derivative), pairing defect, finite-difference scan
  flow      classic RK4 coflow, ragged sets, discrete adjoint with checkpoints
  native    ctypes wrapper of ``ref_engine.c`` (plain C loops for large graphs)
  ds_select power iteration used to fix the integration step

Where the paper is silent, each function's docstring states the reading it
takes; every function here is pinned by the ``-m "not gpu"`` tests against
brute force, closed forms or invariants, except where its docstring says
"parity unpinned".
"""
