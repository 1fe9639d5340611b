"""CPU oracle for HODLR factorization and solve — TEST INFRASTRUCTURE ONLY.

Nothing in the product path may import this package: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` use it.
It is a plain, slow, FP64 NumPy/SciPy restatement of the paper's recursive
algorithm and shares no code, layout or helper with the HIP library.
"""
from .hodlr_oracle import (  # noqa: F401
    Hodlr,
    from_inputs,
    node_range,
    assemble_dense,
    factor,
    solve,
    y_big,
    slogdet,
    transpose,
    solve_adjoint,
    matvec,
    grad_structured,
    logdet_grad_structured,
    loss_and_grads,
    refine,
    low_precision_solver,
    relres,
)
from .extended_sparse import extended_sparse_solve  # noqa: F401
from .construct import KernelSpec, entries as kernel_entries, aca, build as construct_hodlr, dense as kernel_dense  # noqa: F401
