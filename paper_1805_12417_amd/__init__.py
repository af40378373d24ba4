"""MINRES-CG for MI355X: a two-level nested Krylov solver for sparse symmetric
indefinite systems with few negative eigenvalues (outer preconditioned MINRES,
inner CG on the deflated absolute-value preconditioner M_mr = A +
2 V|Lambda|V^T, optionally preconditioned again).

Submodules are imported lazily: `workloads` (seeded inputs) needs no GPU;
`solver` loads the HIP library and raises if it is missing.
"""
__all__ = ["workloads", "solver"]
