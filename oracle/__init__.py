"""FP64 CPU oracle of the coupled phase-field lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import anything from here; the
GPU library and its binding never do.  The oracle shares no code with the GPU
path (own lattice tables, own parameter struct, own arithmetic).

Every function of the oracle is pinned by tests against what the paper and
the mathematics fix (closed forms, invariants, limits), see tests/.
"""
