"""lattice_energies_noalloc against lattice_energies: the same passes with the
partial sums in the library's static scratch, two calls in a row (the second
on a smaller lattice), for each model; the size limit is checked on the host."""
import numpy as np
import pytest

from paper_2006_15122_amd import synth

pytestmark = pytest.mark.gpu


def _lattice(cfg):
    from paper_2006_15122_amd.lattice import Lattice

    return Lattice(cfg, device="cuda:0")


def _same(a, b):
    for k, v in a.items():
        if isinstance(v, float) and np.isnan(v):
            assert np.isnan(b[k]), k
        else:
            assert v == b[k], (k, v, b[k])


@pytest.mark.parametrize("make", [
    lambda N: synth.small(synth.config2(q=100.0), N),
    lambda N: dict(synth.config3(N=N), precision="fp32"),
    lambda N: dict(synth.config_su2u1(N=N), precision="fp32"),
], ids=["scalar", "u1", "su2u1"])
def test_energies_noalloc_matches_energies_on_two_calls(make):
    big, small = _lattice(make(64)), _lattice(make(32))
    big.step(7)
    small.step(5)
    for lat in (big, small):
        ref = lat.energies()
        got = lat.energies_noalloc()
        _same(ref, got)
        # and again after more steps, the scratch keeping the previous call's records
        lat.step(3)
        _same(lat.energies(), lat.energies_noalloc())
    big.close()
    small.close()


def test_energies_noalloc_at_the_largest_scalar_lattice_it_takes():
    # two fields at 512^3: the observation pass writes 32768 records of 13
    # sums, 3.4 MB of the 4 MiB scratch
    cfg = synth.config2(q=100.0, N=512)
    lat = _lattice(cfg)
    lat.step(2)
    _same(lat.energies(), lat.energies_noalloc())
    lat.close()


@pytest.mark.parametrize("cfg", [
    dict(synth.config_su2u1(N=256), precision="fp32", ic="homogeneous"),
    dict(synth.config2(q=100.0, N=640), ic="homogeneous"),
], ids=["su2u1_256", "scalar_640"])
def test_energies_noalloc_rejects_lattices_beyond_its_scratch(cfg):
    from paper_2006_15122_amd.lattice import LatticeError

    # SU(2) x U(1) at 256^3 writes 16 FP64 sums per 256 sites (8 MiB); two
    # fields at 640^3 64000 records of 13 sums (6.7 MB)
    lat = _lattice(cfg)
    with pytest.raises(LatticeError) as e:
        lat.energies_noalloc()
    assert "LAT_ENOMEM" in str(e.value)
    lat.close()
