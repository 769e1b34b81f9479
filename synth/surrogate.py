"""Seeded inputs of the loss surrogate: the sampling workload, random
momenta and frequencies, initial network weights and mini-batch orders.

Everything here is input data shared by the CPU oracle and the GPU path;
no loss function, network output or gradient is computed here.

The surrogate learns Im[-1/eps_LFE](Q, w) over the momentum transfers
Q = q + G and energies that a rate integral sweeps.  For that quantity to
be a function of Q at all, the states must be one band structure evaluated
consistently at k and at k + q: the sampling workload therefore uses the
smooth band model of the generator (energies and coefficients are periodic
smooth functions of k) rather than independent energy draws per q.
"""
from __future__ import annotations

import math

import numpy as np

from .generator import (BASE_SEED, MIXED_CELLS, Workload, _basis_small, fcc_cell, gamma_grid,
                        g_shells, reciprocal_rows)

SURR_SEED = BASE_SEED + 5
N_G = 259                 # G set whose largest |q+G| bounds the query domain
W_MAX_EV = 60.0


def make_surrogate_workload(q_list, kgrid: int = 9, n_g: int = N_G, n_w: int = 16, eta_eV: float = 0.1) -> Workload:
    """Si-like cell of the mixed batch (a = 10.26 bohr, two s and one p shell
    per atom), 4 valence + 6 conduction smooth bands, n^3 k grid, closed G
    shells; q_list gives the momenta whose states are drawn."""
    name, a, species = MIXED_CELLS[1]
    cell = fcc_cell(a, name, species)
    rng = np.random.default_rng(np.random.SeedSequence(BASE_SEED + 3 + 1000 * 1).spawn(3)[2])
    basis = _basis_small(rng, 2, species)
    return Workload(
        name=f"c5_surrogate_{name}", cell=cell, basis=basis, lattice_range=1, n_occ=4, n_bands=10,
        k_frac=gamma_grid(kgrid), G_int=g_shells(cell.lat, n_g),
        w_eV=np.linspace(0.0, W_MAX_EV, n_w), eta_eV=eta_eV, q_list=list(q_list), seed=SURR_SEED,
        energy_ranges=[(4, -12.0, 0.0), (6, 1.1, 15.0)], smooth_bands=True)


def random_q(seed: int, lat: np.ndarray, n: int) -> np.ndarray:
    """n momenta q = f . b with fractional coordinates f uniform in [-1/2, 1/2)^3."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(-0.5, 0.5, size=(n, 3))
    return f @ reciprocal_rows(lat)


def random_w(seed: int, n_q: int, n_w: int, w_max: float = W_MAX_EV) -> np.ndarray:
    """[n_q][n_w] frequencies, uniform in [0, w_max] eV, sorted per q."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.uniform(0.0, w_max, size=(n_q, n_w)), axis=1)


def q_max(wl: Workload) -> float:
    """Largest |G| of the set plus the largest |q| of the sampling cube:
    the radius that bounds every Q = q + G of the data."""
    b = reciprocal_rows(wl.cell.lat)
    g = np.linalg.norm(wl.G_int @ b, axis=1).max()
    corners = np.array([[x, y, z] for x in (-.5, .5) for y in (-.5, .5) for z in (-.5, .5)])
    return float(g + np.linalg.norm(corners @ b, axis=1).max())


def mlp_init(seed: int, widths=(49, 256, 256, 256, 256, 1)) -> np.ndarray:
    """Flat FP32 parameters (W_l row-major then b_l per layer): hidden
    weights N(0, 2/fan_in), output weights N(0, 1/fan_in), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    L = len(widths) - 1
    for i in range(L):
        n_in, n_out = widths[i], widths[i + 1]
        std = math.sqrt((1.0 if i == L - 1 else 2.0) / n_in)
        parts.append(rng.standard_normal(n_out * n_in) * std)
        parts.append(np.zeros(n_out))
    return np.concatenate(parts).astype(np.float32)


def batch_order(seed: int, n_data: int, batch: int, n_epochs: int) -> np.ndarray:
    """Concatenated per-epoch permutations, each cut to whole batches."""
    rng = np.random.default_rng(seed)
    per = (n_data // batch) * batch
    return np.concatenate([rng.permutation(n_data)[:per] for _ in range(n_epochs)]).astype(np.int32)


def holdout_split(seed: int, n: int, frac: float = 0.1):
    """(train indices, held-out indices), a random split of range(n)."""
    p = np.random.default_rng(seed).permutation(n)
    k = int(round(frac * n))
    return np.sort(p[k:]), np.sort(p[:k])
