"""The allocation-free entry point (nepmi_compute_noalloc) against
nepmi_compute: two calls in a row, the second on a smaller batch, each
compared with the allocating entry point on the same inputs.  Both run the
same kernels with the same variants on the same lists, so the results must be
bitwise equal (which implies the parity bars of the evaluation); a batch
beyond the workspace limit must be refused with NEPMI_INVALID_ARG."""
import numpy as np
import pytest

from paper_2607_06969_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_noalloc_matches_compute_on_two_calls():
    from paper_2607_06969_amd import nep
    hp = W.hp_gst()
    m = nep.NepModel(hp, W.random_params(hp, W.SEED_PARAM + 81))
    first = W.concat_systems([W.rocksalt_gst(12, seed=W.SEED_POS + 81),
                              W.amorphous_batch(n_cfg=5, n_min=64, n_max=400, seed=82)])
    second = W.rocksalt_gst(8, seed=W.SEED_POS + 83)   # smaller than the first
    assert second.n_atoms < first.n_atoms
    for s in (first, second):
        b = nep.Batch.from_system(s)
        print(f"[noalloc] N={s.n_atoms} n_cfg={s.n_cfg}", flush=True)
        got = m.compute(b, atom_energy=True, atom_virial=True, noalloc=True)
        ref = m.compute(b, atom_energy=True, atom_virial=True)
        torch.cuda.synchronize()
        for k in ("E", "F", "V", "Ei", "Wi"):
            assert torch.equal(got[k], ref[k]), k
        assert torch.isfinite(got["F"]).all()
        assert float(got["F"].abs().max()) > 0.0


def test_noalloc_rejects_batches_beyond_the_workspace():
    from paper_2607_06969_amd import nep
    from paper_2607_06969_amd._lib import INVALID_ARG, NepmiError
    hp = W.hp_gst()
    m = nep.NepModel(hp, W.random_params(hp, W.SEED_PARAM + 84))
    big = W.rocksalt_gst(40, seed=W.SEED_POS + 84)  # 57,600 atoms: about 120 MiB of work space
    b = nep.Batch.from_system(big)
    with pytest.raises(NepmiError) as e:
        m.compute(b, noalloc=True)
    assert e.value.code == INVALID_ARG
    assert "allocation-free" in str(e.value)
    # the workspace is usable again after the refusal
    small = W.rocksalt_gst(8, seed=W.SEED_POS + 85)
    bs = nep.Batch.from_system(small)
    got = m.compute(bs, noalloc=True)
    ref = m.compute(bs)
    assert torch.equal(got["F"], ref["F"]) and torch.equal(got["E"], ref["E"])
