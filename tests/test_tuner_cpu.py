"""Host side of the layout autotuner: signatures and the cache file."""
import json

from paper_1503_01721_amd import synth


def test_signature_and_cache_lookup(tmp_path, monkeypatch):
    from paper_1503_01721_amd import tuner
    plan = synth.PLANS["cp20_bl20x20_vox32"]
    sig = tuner.signature(plan.n_vox, plan.n_bl, 5070336, "f32", plan.grids, 1)
    assert sig == "vox32768_bl8000_nnz5070336_f32_dg32x32x32_pg20x20x20_rhs1"
    assert tuner.signature(plan.n_vox, plan.n_bl, 5070336, "f16", plan.grids, 1) != sig
    path = tmp_path / "cache.json"
    monkeypatch.setenv(tuner.CACHE_ENV, str(path))
    assert tuner.cache_path() == str(path)
    assert tuner.layout_for(sig) is None                       # no file yet
    path.write_text(json.dumps({sig: {"options": {"dose_tile": [16, 8, 8], "dose_block_rows": 1,
                                                  "price_tile": [4, 2, 8], "panel_cols": 8192}}}))
    opts = tuner.layout_for(sig)
    assert opts == {"dose_tile": (16, 8, 8), "dose_block_rows": 1, "price_tile": (4, 2, 8), "panel_cols": 8192}
    assert tuner.layout_for(sig + "x") is None


def test_committed_cache_names_valid_options():
    """Every cached choice uses knobs the matrix build accepts."""
    from paper_1503_01721_amd import tuner
    allowed = {"dose_tile", "price_tile", "dose_block_rows", "price_block_rows", "panel_cols", "part_entries",
               "dose_layout", "price_layout", "dose_slice_lanes", "price_slice_lanes"}
    for sig, entry in tuner._load(tuner.DEFAULT_CACHE).items():
        assert set(entry["options"]) <= allowed, sig
        assert entry["options"].get("dose_block_rows", 1) in (1, 2, 4)
        for side in ("dose", "price"):
            if entry["options"].get(side + "_layout") == "sliced":
                assert entry["options"].get(side + "_block_rows", 1) == 1
                assert entry["options"].get(side + "_slice_lanes", 8) in (4, 8, 16)
