"""Planted mistakes: each test plants one plausible error in the oracle (on
the CPU, for the duration of the test only) and checks that the pin meant to
catch it fails.  This shows the pins are not vacuous: a dropped Gaussian, a
wrong sign or a missing factor in the oracle would be
caught before it could be trusted against the GPU path."""
import dataclasses
import importlib.util
import os

import numpy as np
import pytest

_spec = importlib.util.spec_from_file_location("oracle_pins", os.path.join(os.path.dirname(__file__),
                                                                           "test_oracle_pins.py"))
pins = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(pins)


def _wrap(monkeypatch, orc, name, change):
    real = getattr(orc, name)
    monkeypatch.setattr(orc, name, lambda *a, **k: change(real(*a, **k)))


def test_the_pins_pass_unplanted(orc):
    pins.test_sog_finite_difference_pressure_and_force(orc)
    pins.test_sog_virial_identity_theorem2(orc)
    pins.test_sog_production_row_error_level(orc)


def test_a_wrong_force_sign_is_caught(orc, monkeypatch):
    def flip(r):
        r = dict(r)
        if r.get("F") is not None:
            F = r["F"].copy()
            F[:, 1] = -F[:, 1]
            r["F"] = F
        return r
    _wrap(monkeypatch, orc, "sog_deterministic", flip)
    with pytest.raises(AssertionError):
        pins.test_sog_finite_difference_pressure_and_force(orc)


def test_a_halved_pressure_is_caught(orc, monkeypatch):
    def halve(r):
        r = dict(r)
        r["P"] = 0.5 * r["P"]  # the full-shell 1/2 applied twice
        return r
    _wrap(monkeypatch, orc, "sog_deterministic", halve)
    with pytest.raises(AssertionError):
        pins.test_sog_virial_identity_theorem2(orc)


def test_a_dropped_gaussian_is_caught(orc, monkeypatch):
    real = orc.sog

    def drop_second(*a, **k):
        p = real(*a, **k)
        wt, w = p.wt.copy(), p.w.copy()
        wt[1] = 0.0  # the term l = 1 (width about 2 sigma) left out of both sums
        w[1] = 0.0
        return dataclasses.replace(p, wt=wt, w=w)
    monkeypatch.setattr(orc, "sog", drop_second)
    with pytest.raises(AssertionError):
        pins.test_sog_production_row_error_level(orc)


def test_a_wrong_sign_in_the_nonradial_estimator_is_caught(orc, monkeypatch):
    def flip(r):
        F, Pr, Pnr, UF = r
        return F, Pr, -Pnr, UF
    _wrap(monkeypatch, orc, "long_range_rb", flip)
    with pytest.raises(AssertionError):
        pins.test_batch_mean_is_unbiased(orc, orc.RECAL_EXCHANGE, 50, 20_000)


def test_transposed_cell_axes_are_caught(orc, monkeypatch):
    def swap_xy(cid):
        # ids built with the x and y strides exchanged: cx n_y + cy instead of cx + n_x cy
        nc = np.array([7, 5, 6])
        cx, cy, cz = cid % nc[0], (cid // nc[0]) % nc[1], cid // (nc[0] * nc[1])
        return cy + nc[1] * (cx + nc[0] * cz)
    _wrap(monkeypatch, orc, "cell_ids", swap_xy)
    with pytest.raises(AssertionError):
        pins.test_cell_ids_contain_their_atoms(orc)
