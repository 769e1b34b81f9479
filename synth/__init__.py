"""Seeded synthetic workloads for the RPA screening path.

This package stands in for the DFT step that, in the paper, supplies Kohn-Sham
coefficients and energies (Sec. III).  It draws cells, Gaussian shells, grids
and Lowdin-orthonormal random states from fixed seeds, and is the only code
shared by the CPU oracle and the HIP path.  It computes no pair density, no
response function and no dielectric matrix.
"""
from .generator import (  # noqa: F401
    HARTREE_EV,
    Cell,
    Basis,
    Workload,
    QStates,
    make_smallest,
    make_si_ng113,
    make_mixed_batch_items,
    make_all_electron,
    make_tiny,
    fcc_cell,
    reciprocal_rows,
    gamma_grid,
    g_cube,
    g_shells,
    draw_states,
)
