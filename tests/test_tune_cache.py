"""Host logic of the autotuner's table and cache file (no GPU): parsing,
architecture filter, bucketing of right-hand-side counts, defaults."""
import pytest


@pytest.fixture
def P():
    import paper_2104_04609_amd as P
    P.tune_clear()
    yield P
    P.tune_clear()


LINES = [
    "bem-tune-v1 gfx950 T=20480 R=4 block=128 multi=4 gemm_min=8 skinny_min=4 path=1 t_mf=0.05 t_dense=0.002 t_asm=0.09",
    "bem-tune-v1 gfx950 T=20480 R=1 block=256 multi=1 gemm_min=2 path=0 t_mf=0.0225 t_dense=0 t_asm=0",
    "bem-tune-v1 gfx942 T=20480 R=1 block=64 multi=1 gemm_min=2 path=1 t_mf=1 t_dense=1 t_asm=1",
    "bem-tune-v1 gfx950 T=1280 R=3 block=64 multi=2 gemm_min=4 path=0 t_mf=1 t_dense=0 t_asm=0",
    "bem-tune-v1 gfx950 T=1280 R=2 block=96 multi=2 gemm_min=4 path=0 t_mf=1 t_dense=0 t_asm=0",
    "bem-tune-v1 gfx950 T=1280 R=2 block=64 multi=2 gemm_min=4 path=7 t_mf=1 t_dense=0 t_asm=0",
    "garbage line",
    "bem-tune-v1 gfx950 T=1280 R=2 block=64 multi=2",
    "bem-tune-v1 gfx950 T=5120 R=16 block=64 multi=4 gemm_min=16 path=1 t_mf=2 t_dense=0.1 t_asm=0.3",
]


def test_cache_load_and_lookup(P, tmp_path):
    f = tmp_path / "tune.txt"
    f.write_text("\n".join(LINES) + "\n")
    n = P.tune_cache_load(str(f), "gfx950")
    assert n == 3   # R=3 is not a bucket; block=96, path=7 and short lines rejected
    e, tuned = P.tune_lookup(20480, 5)   # bucket 4..7
    assert tuned and e["block"] == 128 and e["multi"] == 4 and e["path"] == 1
    assert e["skinny_min"] == 4
    assert e["t_assembly"] == pytest.approx(0.09)
    e, tuned = P.tune_lookup(20480, 1)
    assert tuned and e["path"] == 0 and e["t_matrix_free"] == pytest.approx(0.0225)
    assert e["skinny_min"] == 24   # absent from the line: default
    e, tuned = P.tune_lookup(5120, 40)   # bucket 16+
    assert tuned and e["gemm_min"] == 16
    e, tuned = P.tune_lookup(1280, 2)
    assert not tuned and e["path"] == -1
    assert e["block"] == P.tune_get("farfield.block")
    assert e["multi"] == P.tune_get("farfield.multi_max")


def test_later_lines_win_and_missing_file(P, tmp_path):
    f = tmp_path / "t.txt"
    f.write_text(LINES[1] + "\n" + LINES[1].replace("block=256", "block=64") + "\n")
    assert P.tune_cache_load(str(f), "gfx950") == 2
    assert P.tune_lookup(20480, 1)[0]["block"] == 64
    P.tune_clear()
    assert not P.tune_lookup(20480, 1)[1]
    assert P.tune_cache_load(str(tmp_path / "absent.txt"), "gfx950") == 0


def test_tune_knob_validation(P):
    with pytest.raises(P.BemError):
        P.tune_set("farfield.block", 100)
    with pytest.raises(P.BemError):
        P.tune_set("no.such.key", 1)
    old = P.tune_get("farfield.block")
    P.tune_set("farfield.block", 128)
    assert P.tune_lookup(999, 1)[0]["block"] == 128
    P.tune_set("farfield.block", old)
