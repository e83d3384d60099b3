"""Pins of the closed-form bounds against the numbers printed in Sec. 4.3 and
Sec. 4.4."""

import json
import os

import numpy as np
import pytest

from oracle import theory
from oracle.grid import Grid

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")))
C_HAT = 1.0 + 0.2 ** 2


def test_bounded_stiffness_numbers():
    gold = GOLD["bounded_stiffness"]
    for n in (32, 64, 128, 256):
        g = Grid(n, n, 1, lengths=(1.0, 2 * np.pi, 2 * np.pi))
        k = gold["k_times_N2"] / n ** 2
        beta = theory.beta_n(0.2, 1.0, k, C_HAT, g.max_symbol())
        assert beta == pytest.approx(gold["h_max"], abs=5e-5)
        qh = theory.q_bar(0.5, 0.2, beta)
        assert qh == pytest.approx(gold["q_H"], abs=5e-5)
        th = theory.vartheta2(qh, theory.gamma_m(0.5, 1.0))
        assert th == pytest.approx(gold["vartheta2"], abs=5e-5)
        assert theory.explicit_limit_ratio(k, C_HAT, g.max_symbol(), 0.2) == pytest.approx(gold["explicit_limit_ratio"], abs=5e-3)
        assert k * C_HAT * g.max_symbol() == pytest.approx(gold["k_Chat_max_symbol"], abs=5e-5)
        assert beta / 0.2 == pytest.approx(gold["condition_number"], abs=0.05)


def test_fixed_k_vartheta2_and_lambda_bd():
    gold = GOLD["fixed_k_vartheta2"]
    g = Grid(gold["N"], gold["N"], 1, lengths=(1.0, 2 * np.pi, 2 * np.pi))
    beta = theory.beta_n(0.2, 1.0, gold["dt"], C_HAT, g.max_symbol())
    th = theory.vartheta2(theory.q_bar(0.5, 0.2, beta), theory.gamma_m(0.5, 1.0))
    assert th == pytest.approx(gold["vartheta2"], abs=5e-5)
    lb = GOLD["lambda_bd"]
    for n, ref in zip(lb["N"], lb["lambda_bd"]):
        g = Grid(n, n, 1, lengths=(1.0, 2 * np.pi, 2 * np.pi))
        beta = theory.beta_n(0.2, 1.0, 1e-2, C_HAT, g.max_symbol())
        assert theory.lambda_bd(0.2, beta) == pytest.approx(ref, abs=5e-3)


def test_iteration_bound_monotone():
    assert theory.iteration_bound(1.0, 0.9574, 1e-8) == 2 * int(np.ceil(np.log(1e8) / np.log(1 / 0.9574)))
    assert theory.kappa(0.5, 1.0, 1.0) == 1.0
    assert theory.gamma_m(0.5, 1.0) == pytest.approx(2 * 0.5 / 1.25)
