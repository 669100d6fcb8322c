"""hsm_stencils_export_noalloc (device temporaries from the library's fixed
scratch array, no allocation) against hsm_stencils_export: identical classes,
offsets, indices and weights, on two calls in a row with the second set
smaller than the first (the array keeps the first call's contents), and a set
too large for the array is refused."""
import numpy as np
import pytest
import torch

from paper_2303_01760_amd import nodegen as ng

pytestmark = pytest.mark.gpu


def _build(s, m):
    from paper_2303_01760_amd import hsm
    dev = torch.device("cuda")
    return hsm.build_stencils(torch.tensor(s.x, device=dev), torch.tensor(s.kind, device=dev),
                              torch.tensor(s.normal, device=dev), s.h, m)


def test_export_noalloc_matches_export_on_two_calls():
    sets = [(ng.obstacles2d(h=0.005, n_obst=8, seed=41), 4), (ng.cavity2d(h=0.05), 2)]
    assert sets[1][0].n < sets[0][0].n
    for s, m in sets:
        st = _build(s, m)
        ref = st.export()
        got = st.export(noalloc=True)
        for key in ("cls", "off", "idx", "w"):
            assert np.array_equal(got[key], ref[key]), (s.name, key)
        print(f"{s.name}: N={s.n} nnz={len(ref['idx'])} export_noalloc identical")


def test_export_noalloc_refuses_sets_beyond_its_array():
    from paper_2303_01760_amd import hsm
    s = ng.obstacles2d(h=0.002)
    st = _build(s, 4)
    info = st.info()
    need = 4 * s.n + 8 * (s.n + 1) + (4 + 8 * (s.d + 2)) * info["nnz"]
    assert need > 64 << 20, need
    with pytest.raises(hsm.HsmError) as e:
        st.export(noalloc=True)
    assert e.value.code == hsm.E_INVALID
    assert "scratch" in str(e.value)
    # the ordinary export still serves it
    assert len(st.export()["idx"]) == info["nnz"]
