"""The constants that the paper prints for its halo example and its q-space
binning (tests/golden/halo_and_binning.txt, each line citing where the paper
gives it) against what the oracle's rate integral and the library binding
use: the halo speeds and density of oracle/rates.py, their values in units
of c as the paper rounds them, and the binning defaults of QBins."""
import inspect
import os

import pytest

from oracle import rates

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "halo_and_binning.txt")


def _golden():
    vals = {}
    for line in open(GOLDEN):
        line = line.split("|")[0].strip()
        if not line or line.startswith("#"):
            continue
        name, value, _unit = line.split()[:3]
        vals[name] = float(value)
    return vals


def test_halo_parameters_as_printed():
    g = _golden()
    assert rates.HALO["vesc"] == g["v_escape_kms"]
    assert rates.HALO["vE"] == g["v_earth_kms"]
    assert rates.HALO["rho_chi"] == g["rho_chi"]
    # the same speeds in units of c, rounded to the paper's four decimals
    c = rates.C_KMS
    assert round(rates.HALO["vesc"] / c, 4) == g["v_escape_c"]
    assert round(rates.HALO["vE"] / c, 4) == g["v_earth_c"]
    assert round((rates.HALO["vesc"] + rates.HALO["vE"]) / c, 4) == g["v_max_c"]


def test_alpha_me_is_inverse_bohr():
    """Momenta in units of alpha m_e equal momenta in bohr^-1 (the binding's
    and the oracle's unit for dq): alpha m_e c = hbar / a_0."""
    assert rates.AME_EV == pytest.approx(rates.ALPHA * rates.ME_EV, rel=1e-15)
    # hbar c / a_0 in eV from CODATA: 197.3269804 eV nm / 0.0529177210903 nm
    assert rates.AME_EV == pytest.approx(197.3269804 / 0.0529177210903, rel=1e-8)


def test_binning_defaults_as_printed():
    from paper_2603_12326_amd.qcx import QBins

    g = _golden()
    p = inspect.signature(QBins.__init__).parameters
    assert p["n_theta"].default == g["n_theta"]
    assert p["n_phi"].default == g["n_phi"]
    assert p["dq"].default == g["dq"]
