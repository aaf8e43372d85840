"""Index files written by the library (no GPU needed): the record layout of
paper section 3 (vector, then R int32 ids, in a fixed slot), meta.json, and
ann_build_index's graph equal to the input generator's for the same seed."""
import json
import os

import numpy as np
import pytest

import synth


def _lib_or_skip():
    from paper_2507_10070_amd import flashann

    if not os.path.exists(flashann.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    return flashann


@pytest.mark.parametrize("dtype,d,R,slot", [("u8", 128, 64, 512), ("i8", 100, 48, 512),
                                            ("f32", 96, 16, 448), ("u8", 7, 3, 32)])
def test_save_index_layout(tmp_path, dtype, d, R, slot):
    fl = _lib_or_skip()
    base = synth.make_base(300, d, dtype, 4, 11)
    rng = np.random.default_rng(3)
    adj = rng.integers(-1, 300, size=(300, R)).astype(np.int32)
    p = str(tmp_path / "ix")
    fl.save_index(p, base, adj, 17, slot)
    meta = json.load(open(os.path.join(p, "meta.json")))
    assert meta == {"format": "flashann-1", "n": 300, "d": d, "dtype": dtype, "R": R,
                    "entry": 17, "slot_bytes": slot}
    vec = np.fromfile(os.path.join(p, "vectors.bin"), dtype=base.dtype).reshape(300, d)
    np.testing.assert_array_equal(vec, base)
    rec = np.fromfile(os.path.join(p, "records.bin"), dtype=np.uint8).reshape(300, slot)
    vb = d * base.dtype.itemsize
    vp = (vb + 15) // 16 * 16
    np.testing.assert_array_equal(rec[:, :vb], base.view(np.uint8).reshape(300, vb))
    assert (rec[:, vb:vp] == 0).all()
    ids = rec[:, vp:vp + 4 * R].copy().view(np.int32)
    np.testing.assert_array_equal(ids, adj)
    assert (rec[:, vp + 4 * R:] == 0).all()


def test_save_index_rejects_small_slot(tmp_path):
    fl = _lib_or_skip()
    base = np.zeros((10, 16), np.uint8)
    adj = np.zeros((10, 4), np.int32)
    with pytest.raises(fl.AnnError) as e:
        fl.save_index(str(tmp_path / "x"), base, adj, 0, 16)
    assert e.value.code == -22


def test_build_index_graph_is_the_generators(tmp_path):
    fl = _lib_or_skip()
    base = synth.make_base(3000, 32, "u8", 6, 21)
    p = str(tmp_path / "ix")
    fl.build_index(p, base, 12, 96, 777)
    adj, entry = synth.build_graph(base, 12, 777)
    meta = json.load(open(os.path.join(p, "meta.json")))
    assert meta["entry"] == entry
    rec = np.fromfile(os.path.join(p, "records.bin"), dtype=np.uint8).reshape(3000, 96)
    np.testing.assert_array_equal(rec[:, 32:32 + 48].copy().view(np.int32), adj)
