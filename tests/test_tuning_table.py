"""The process-wide launch-shape table (host only: no device is touched)."""
import os

import pytest

import paper_1807_10151_amd as sp


@pytest.fixture()
def clean():
    sp.tuning_clear()
    yield
    sp.tuning_clear()


def test_set_list_erase(clean):
    g = sp.Geometry(64, 64, 90, 91)
    h = sp.Geometry(37, 53, 45, 61, pixel=0.7, theta0=0.1, dtheta=0.05, bin_spacing=0.9, bin_offset=0.2)
    sp.tuning_set(g, 2, 4)
    sp.tuning_set(h, 8, 2)
    sp.tuning_set(g, 4, 2)                      # replaces g's entry
    got = {tuple(vars(k).values()): (p, x) for k, p, x in sp.tuning_list()}
    assert got == {tuple(vars(g).values()): (4, 2), tuple(vars(h).values()): (8, 2)}
    sp.tuning_set(g, 0, 0)
    assert [k for k, _, _ in sp.tuning_list()] == [h]


@pytest.mark.parametrize("parts,px", [(0, 2), (9, 2), (3, 3), (1, 1), (-1, 4)])
def test_rejects_bad_shapes(clean, parts, px):
    with pytest.raises(sp.SupPCGError):
        sp.tuning_set(sp.Geometry(16, 16, 8, 24), parts, px)
    assert sp.tuning_list() == []


def test_rejects_invalid_geometry(clean):
    with pytest.raises(sp.SupPCGError):
        sp.tuning_set(sp.Geometry(16, 16, 0, 24), 1, 2)


def test_json_roundtrip(clean, tmp_path):
    gs = [sp.Geometry(512, 512, 720, 725), sp.Geometry(243, 243, 360, 345, pixel=0.0752, bin_spacing=0.0752)]
    sp.tuning_set(gs[0], 1, 4)
    sp.tuning_set(gs[1], 2, 2)
    path = os.path.join(tmp_path, "shapes.json")
    sp.tuning_save(path)
    sp.tuning_clear()
    assert sp.tuning_list() == []
    sp.tuning_load(path)
    assert sorted(((k.rows, p, x) for k, p, x in sp.tuning_list())) == [(243, 2, 2), (512, 1, 4)]
    assert {k for k, _, _ in sp.tuning_list()} == set(gs)
