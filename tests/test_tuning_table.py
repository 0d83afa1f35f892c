"""The committed tuning table: well formed, every entry accepted by the library's own
validation (spm_tuning_set, host only), and one signature per problem class and element
type, so a float32 and a bfloat16 batch never share an entry (kinds: pipeline, batch, insert, transpose)."""
import json
import os

from paper_1805_03380_amd import _lib, autotune


def _lib_or_build():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1805_03380_amd import build
        build.build()
    return _lib.load()


def test_table_entries_are_valid_tunings():
    _lib_or_build()
    with open(autotune.DEFAULT_TABLE) as f:
        table = json.load(f)
    assert table, "empty tuning table"
    saved = _lib.get_tuning().as_dict()
    try:
        for dev, entries in table.items():
            arch, _, ver = dev.partition("|")
            assert arch.split(":")[0].startswith("gfx") and arch.endswith("cu"), dev
            assert ver, dev
            for sig, entry in entries.items():
                kind = sig.split(":")[0]
                assert kind in ("pipeline", "batch", "insert", "transpose"), sig
                assert entry["tuning"] and all(ms > 0 for ms in entry["ms"].values()), sig
                _lib.set_tuning(**entry["tuning"])  # raises on a value the library refuses
                got = _lib.get_tuning().as_dict()
                assert all(got[k] == v for k, v in entry["tuning"].items()), sig
    finally:
        _lib.set_tuning(**saved)


def test_signatures_separate_element_types_and_sizes():
    f32 = autotune.batch_signature("float32")
    bf16 = autotune.batch_signature("bfloat16")
    assert f32 != bf16 and f32.endswith("float32:float32") and bf16.endswith("bfloat16:bfloat16")
    a = autotune.signature("pipeline", 10**6, 10**6, 2 * 10**7, 128, "float32", "float32")
    b = autotune.signature("pipeline", 10**5, 10**5, 10**6, 64, "float32", "float32")
    c = autotune.signature("pipeline", 10**5, 10**5, 10**6, 64, "float64", "float32")
    assert len({a, b, c}) == 3
    assert a == "pipeline:r20:c20:n24:k128:float32:float32"
