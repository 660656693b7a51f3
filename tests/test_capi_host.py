"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/sse.h declares, rejects bad descriptors before
touching a device, and its host alias table equals the oracle's."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2509_05047_amd as sse
import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "sse.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sse_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert len(names) >= 22
    lib = sse.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(sse.SIGNATURES), set(names) ^ set(sse.SIGNATURES)


def test_abi_version():
    assert sse.lib().sse_abi_version() == 1


def test_structure_sizes_match_header_layout():
    assert C.sizeof(sse.ScannerDesc) == 28
    assert C.sizeof(sse.SinoDesc) == 24
    assert C.sizeof(sse.PhysicsDesc) == 40
    assert C.sizeof(sse.PhantomDesc) == 36
    assert C.sizeof(sse.LutDesc) == 28
    assert C.sizeof(sse.Outputs) == 56
    assert C.sizeof(sse.ServerCfg) == 32
    assert C.sizeof(sse.Request) == 48
    assert C.sizeof(sse.Completion) == 64
    assert C.sizeof(sse.ServerStats) == 72
    assert C.sizeof(sse.GapDesc) == 24
    assert C.sizeof(sse.KernelTiming) == 32
    assert C.sizeof(sse.EdgeGeom) == 24


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_host_alias_table_equals_oracle(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 3000))
    act = rng.uniform(0, 3, n).astype(np.float32)
    act[rng.random(n) < 0.4] = 0.0
    act[int(rng.integers(0, n))] = 1.0
    th, al = sse.build_alias_table(act)
    oth, oal = O.build_alias(act)
    assert np.array_equal(th, oth) and np.array_equal(al, oal)


@pytest.mark.parametrize("kind", ["few_heavy", "one_hot", "uniform", "heavy_last", "ragged_threads"])
def test_host_alias_table_equals_oracle_on_skewed_activity(kind):
    """Pairing extremes: a few heavy voxels among many empty ones (one large
    column pairs with long runs of small ones), a single active voxel, all
    masses equal (no pairing at all), the heavy voxel last, and a size past
    the threaded quantisation's threshold with ranges of unequal length."""
    rng = np.random.default_rng(5)
    if kind == "few_heavy":
        act = np.zeros(5000, np.float32)
        act[rng.choice(5000, 7, replace=False)] = rng.uniform(1, 100, 7).astype(np.float32)
    elif kind == "one_hot":
        act = np.zeros(777, np.float32)
        act[400] = 2.5
    elif kind == "uniform":
        act = np.full(1024, 0.75, np.float32)
    elif kind == "heavy_last":
        act = rng.uniform(0, 1, 2000).astype(np.float32)
        act[-1] = 1e4
    else:
        n = (1 << 20) + 12345
        act = rng.uniform(0, 2, n).astype(np.float32)
        act[rng.random(n) < 0.5] = 0.0
    th, al = sse.build_alias_table(act)
    oth, oal = O.build_alias(act)
    assert np.array_equal(th, oth) and np.array_equal(al, oal)


def test_host_alias_table_equals_oracle_on_clinical_phantom():
    _, _, act = W.clinical_body()
    th, al = sse.build_alias_table(act)
    oth, oal = O.build_alias(act)
    assert np.array_equal(th, oth) and np.array_equal(al, oal)


def test_alias_table_rejects_bad_activity():
    with pytest.raises(sse.SseError) as e:
        sse.build_alias_table(np.zeros(5, np.float32))
    assert e.value.status == sse.EINVAL
    with pytest.raises(sse.SseError):
        sse.build_alias_table(np.array([1.0, np.inf], np.float32))


def _create(scanner, sino, physics):
    h = C.c_void_p()
    sc, sn, ph = sse.scanner_desc(scanner), sse.sino_desc(sino), sse.physics_desc(physics)
    return sse.lib().sse_create(C.byref(h), 0, C.byref(sc), C.byref(sn), C.byref(ph))


@pytest.mark.parametrize("mutate", [
    lambda s, n, p: setattr(s, "n_crystals", 63),
    lambda s, n, p: setattr(n, "n_view", 31),
    lambda s, n, p: setattr(n, "n_plane", 8),
    lambda s, n, p: setattr(n, "n_rad", 62),
    lambda s, n, p: setattr(n, "n_rad", 65),
    lambda s, n, p: setattr(n, "tof_bin_mm", 0.0),
    lambda s, n, p: p.update(rayleigh_beta=0.0),
    lambda s, n, p: p.update(e_lo_kev=700.0),
    lambda s, n, p: p.update(max_interactions=0),
    lambda s, n, p: p.update(e_kill_kev=50.0),   # below the binary32 energy model's range
    lambda s, n, p: p.update(f_compton=-1.0),
])
def test_create_rejects_bad_descriptors(mutate):
    w = W.WORKLOADS["tiny"]
    s = W.Scanner(**w.scanner.__dict__)
    n = W.Sinogram(**w.sino.__dict__)
    p = dict(w.physics)
    mutate(s, n, p)
    assert _create(s, n, p) == sse.EINVAL
    assert sse.lib().sse_last_error() != b""


# --------------------------------------------------------------------------
# edge-crystal LUT (host helper): the library's own Eq. (1)-(3) against the
# oracle's (two independent implementations of the same reading)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["transaxial", "axial"])
def test_edge_lut_equals_oracle(which):
    gt, ga = W.edge_geometries(W.signa_scanner(), W.SIGNA_GAPS)
    g = gt if which == "transaxial" else ga
    lib_lut = sse.build_edge_lut(g)
    orc_lut = O.edge_lut(g)
    assert lib_lut.shape == orc_lut.shape == (W.EDGE_N_ANGLE, W.EDGE_N_POS)
    assert np.abs(lib_lut.astype(np.float64) - orc_lut).max() < 2e-7


def test_edge_lut_equals_oracle_on_odd_bins():
    g = dict(gap_mm=3.5, depth_mm=20.0, doi_mm=6.0, mu_per_mm=0.12, n_angle=37, n_pos=5)
    assert np.abs(sse.build_edge_lut(g).astype(np.float64) - O.edge_lut(g)).max() < 2e-7


@pytest.mark.parametrize("bad", [dict(n_angle=0), dict(n_pos=-1), dict(gap_mm=0.0), dict(depth_mm=-1.0),
                                 dict(doi_mm=30.0), dict(mu_per_mm=0.0), dict(gap_mm=float("nan"))])
def test_edge_lut_rejects_bad_geometry(bad):
    g = dict(gap_mm=3.0, depth_mm=25.0, doi_mm=8.0, mu_per_mm=0.087, n_angle=36, n_pos=16)
    g.update(bad)
    with pytest.raises(sse.SseError) as e:
        sse.build_edge_lut(g)
    assert e.value.status == sse.EINVAL


def test_pair_pruning_rejects_null_context():
    assert sse.lib().sse_set_pair_pruning(None, 1) == sse.EINVAL
    assert sse.lib().sse_set_pair_buffer(None, 1 << 27) == sse.EINVAL
