"""Reference oracle for the stress-transfer hot path (TEST INFRASTRUCTURE ONLY).

A plain, slow, FP64 CPU implementation of what the HIP library computes, written
from the paper (Ciardo & Romanet, "A divide-and-conquer strategy for fast
elastodynamic simulation of earthquakes and aseismic slip on fault networks"):

* ``geometry``      fault discretisation and the minimum time step (Sections 2.3.1, 3.1)
* ``interaction``   closed-form antiplane primitives, the space-time kernel, causality
                    windows, static dipole tail, dense uncompressed interaction sum
                    (Section 2.3.2, eqs. for the discretised interactions and primitives)
* ``selfterm``      non-replicating spectral self term: mode kernel K(n,t), its cell
                    integrals, mode-dependent windows, explicit DFT (Section 2.3.1)
* ``friction``      rate-and-state strength, intermediate/aging state law, Newton solve
                    (Section 2.2, Section 2.4)
* ``hpartition``    per-fault binary cluster trees, bounding circles, admissibility,
                    dual-tree traversal (Section 2.3.2, H-matrix paragraphs)
* ``seas``          prescribed-history evaluation and the predictor-corrector step
                    (Section 2.4)

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg may
import or run anything here.  It shares no code with the HIP path; both read the
seeded inputs of ``seas_inputs``.

Parity status: every function is pinned by a ``-m "not gpu"`` test against values the
paper prints, closed forms, invariants or brute force, except the full SEAS trajectory
composition beyond one step, which is pinned only through its parts (the paper shows
trajectories as plots only).
"""
