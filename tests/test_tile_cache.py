"""The autotune cache file of the Python binding: keys and file handling
(no GPU needed)."""
import json

import paper_2511_15269_amd as fmm


def test_key_names_every_part_of_the_choice():
    prm = fmm.params(p=8, leaf_max=128, splits=3, theta=0.8, precision="fp64", max_rhs=1)
    k = fmm.tile_cache_key("gfx950:sramecc+:xnack-", prm, 1 << 20)
    assert k == "gfx950|p8|fp64|R1|s3|leaf128|theta0.8|cross|single|n2^20"
    assert fmm.tile_cache_key("gfx950", prm, 1 << 20) == k
    other = [fmm.tile_cache_key("gfx942", prm, 1 << 20),
             fmm.tile_cache_key("gfx950", fmm.params(p=7, leaf_max=128, splits=3, theta=0.8), 1 << 20),
             fmm.tile_cache_key("gfx950", fmm.params(p=8, leaf_max=128, splits=3, theta=0.8,
                                                     precision="fp32"), 1 << 20),
             fmm.tile_cache_key("gfx950", prm, 1 << 18),
             fmm.tile_cache_key("gfx950", prm, 1 << 20, "multi"),
             fmm.tile_cache_key("gfx950", fmm.params(p=8, leaf_max=128, splits=3, theta=0.8,
                                                     lists="same"), 1 << 20)]
    assert len(set(other + [k])) == len(other) + 1


def test_write_then_read_round_trip(tmp_path):
    path = str(tmp_path / "tiles.json")
    assert fmm.read_tile_cache(path) == {}
    t = {"p2p_groups": 2, "leaves_per_wave": 2, "m2l_waves": 1, "chain_waves": 4,
         "near_stream": 2, "batch_p2p_waves": 4, "unrelated": 9}
    fmm.write_tile_cache(path, "a", t)
    fmm.write_tile_cache(path, "b", dict(t, p2p_groups=4))
    got = fmm.read_tile_cache(path)
    assert got["a"] == {k: t[k] for k in fmm.__dict__["TILE_FIELDS"]}
    assert got["b"]["p2p_groups"] == 4
    assert sorted(p.name for p in tmp_path.iterdir()) == ["tiles.json"]  # no temporaries left


def test_unreadable_files_count_as_empty(tmp_path):
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert fmm.read_tile_cache(str(bad)) == {}
    lst = tmp_path / "list.json"
    lst.write_text(json.dumps([1, 2]))
    assert fmm.read_tile_cache(str(lst)) == {}
    fmm.write_tile_cache(str(bad), "k", {"p2p_groups": 1})
    assert fmm.read_tile_cache(str(bad)) == {"k": {"p2p_groups": 1}}
