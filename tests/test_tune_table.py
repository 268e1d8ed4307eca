"""CPU checks of the tuning table (pf_tune_set, pf_tune_load, pf_tune_lookup,
PF_FLAG_TUNED argument rules) and of the table file the package ships: every
call here is host-only."""
import os

import pytest

import paper_2308_00763_amd as pf
from paper_2308_00763_amd import tune


@pytest.fixture
def table():
    """An empty table for the test; the shipped one is reinstalled after."""
    pf.pf_tune_clear()
    yield
    pf.pf_tune_clear()
    if os.path.exists(pf.TUNE_TABLE):
        pf.pf_tune_load(pf.TUNE_TABLE)


def test_empty_table_resolves_to_the_defaults(table):
    assert pf.pf_tune_lookup("gfx950", "f16", 1 << 20) == (0, 0)


def test_lookup_takes_the_bucket_else_the_nearest_one(table):
    pf.pf_tune_set("gfx950", "f16", 12, 512, 128)
    pf.pf_tune_set("gfx950", "f16", 16, 128, 1024)
    pf.pf_tune_set("gfx950", "f32", 14, 256, 64)
    pf.pf_tune_set("gfx942", "f16", 14, 512, 512)
    # bucket = ceil(log2 N)
    assert tune.bucket(4096) == 12 and tune.bucket(4097) == 13 and tune.bucket(1) == 0
    assert pf.pf_tune_lookup("gfx950", "f16", 4096) == (512, 128)      # bucket 12
    assert pf.pf_tune_lookup("gfx950", "f16", 3000) == (512, 128)      # 12
    assert pf.pf_tune_lookup("gfx950", "f16", 1 << 16) == (128, 1024)  # 16
    assert pf.pf_tune_lookup("gfx950", "f16", 1) == (512, 128)         # 0: nearest is 12
    assert pf.pf_tune_lookup("gfx950", "f16", 1 << 24) == (128, 1024)  # 24: nearest is 16
    assert pf.pf_tune_lookup("gfx950", "f16", 5000) == (512, 128)      # 13: 12 is nearer
    assert pf.pf_tune_lookup("gfx950", "f16", 1 << 14) == (512, 128)   # 14: tie, the smaller bucket
    assert pf.pf_tune_lookup("gfx950", "f16", (1 << 14) + 1) == (128, 1024)  # 15: 16 is nearer
    # other dtypes and architectures have their own entries
    assert pf.pf_tune_lookup("gfx950", "f32", 1 << 20) == (256, 64)
    assert pf.pf_tune_lookup("gfx942", "f16", 100) == (512, 512)
    assert pf.pf_tune_lookup("gfx950", "bf16", 1 << 20) == (0, 0)
    assert pf.pf_tune_lookup("gfx90a", "f16", 1 << 20) == (0, 0)
    # an entry with the same key replaces the old one
    pf.pf_tune_set("gfx950", "f16", 12, 0, 256)
    assert pf.pf_tune_lookup("gfx950", "f16", 4096) == (0, 256)


@pytest.mark.parametrize("args", [
    ("", "f16", 12, 256, 256), ("gfx950:sramecc+", "f16", 12, 256, 256), ("g" * 32, "f16", 12, 256, 256),
    ("gfx950", 7, 12, 256, 256), ("gfx950", "f16", -1, 256, 256), ("gfx950", "f16", 29, 256, 256),
    ("gfx950", "f16", 12, 64, 256), ("gfx950", "f16", 12, 1024, 256), ("gfx950", "f16", 12, 300, 256),
    ("gfx950", "f16", 12, 256, 32), ("gfx950", "f16", 12, 256, 2048), ("gfx950", "f16", 12, 256, 96)])
def test_bad_entries_are_rejected(table, args):
    with pytest.raises(pf.PfError) as ei:
        pf.pf_tune_set(*args)
    assert ei.value.code == pf.PF_ERR_INVALID_ARG
    assert pf.pf_tune_lookup("gfx950", "f16", 4096) == (0, 0)


def test_load_reads_entries_and_comments(table, tmp_path):
    path = tmp_path / "t.txt"
    path.write_text("# a comment\n\ngfx950 f16 20 512 0   # trailing comment\n"
                    "  gfx950 bf16 20 0 1024\n" "gfx950 f64 10 128 64\n")
    assert pf.pf_tune_load(str(path)) == 3
    assert pf.pf_tune_lookup("gfx950", "f16", 1 << 20) == (512, 0)
    assert pf.pf_tune_lookup("gfx950", "bf16", 1 << 20) == (0, 1024)
    assert pf.pf_tune_lookup("gfx950", "f64", 1000) == (128, 64)


@pytest.mark.parametrize("bad", ["gfx950 f16 20 512", "gfx950 f16 20 512 0 7", "gfx950 fp16 20 512 0",
                                 "gfx950 f16 20 500 0", "gfx950 f16 40 512 0", "gfx950 f16 x 512 0"])
def test_a_bad_line_installs_nothing(table, tmp_path, bad):
    path = tmp_path / "t.txt"
    path.write_text("gfx950 f32 20 512 0\n" + bad + "\n")
    with pytest.raises(pf.PfError) as ei:
        pf.pf_tune_load(str(path))
    assert ei.value.code == pf.PF_ERR_INVALID_ARG and ":2:" in pf.pf_last_error()
    assert pf.pf_tune_lookup("gfx950", "f32", 1 << 20) == (0, 0)


def test_missing_file_is_an_error(table, tmp_path):
    with pytest.raises(pf.PfError):
        pf.pf_tune_load(str(tmp_path / "none.txt"))


def test_lookup_argument_errors(table):
    for args in (("", "f16", 10), ("gfx950", 9, 10), ("gfx950", "f16", 0)):
        with pytest.raises(pf.PfError):
            pf.pf_tune_lookup(*args)


def test_tuned_flag_rules():
    ok = pf.make_params(5000, 128, 128, "f16", tuned=True)
    assert pf.pf_workspace_bytes(ok) == pf.pf_workspace_bytes(pf.make_params(5000, 128, 128, "f16"))
    for bad in (dict(threads_a=512), dict(threads_c=128), dict(naive_half=True)):
        p = pf.make_params(5000, 128, 128, "f16", tuned=True, **bad)
        with pytest.raises(pf.PfError) as ei:
            pf.pf_workspace_bytes(p)
        assert ei.value.code == pf.PF_ERR_INVALID_ARG


def test_batches_take_tuned_and_sized_members_but_no_other_variant():
    ps = [pf.make_params(5000, 128, 128, "f16", tuned=True), pf.make_params(70001, 128, 128, "f16", threads_a=512),
          pf.make_params(3000, 128, 128, "f16", threads_a=128, threads_c=1024),
          pf.make_params(1000, 128, 128, "f16", diagnostics=True)]
    assert pf.pf_batch_workspace_bytes(ps) > 0
    for bad in (dict(naive_likelihood=True), dict(naive_resample=True), dict(naive_half=True),
                dict(metropolis_steps=8)):
        with pytest.raises(pf.PfError):
            pf.pf_batch_workspace_bytes(ps + [pf.make_params(1000, 128, 128, "f16", **bad)])


def test_shipped_table_parses_and_covers_every_dtype():
    assert os.path.exists(pf.TUNE_TABLE)
    rows = []
    for line in open(pf.TUNE_TABLE):
        line = line.split("#", 1)[0].split()
        if line:
            rows.append(line)
    assert rows
    assert {r[1] for r in rows} == set(tune.TABLE_DTYPES)
    assert {int(r[2]) for r in rows} == set(tune.TABLE_BUCKETS)
    pf.pf_tune_clear()
    try:
        assert pf.pf_tune_load(pf.TUNE_TABLE) == len(rows)
        for arch, dt, b, ta, tc in rows:
            assert pf.pf_tune_lookup(arch, dt, 1 << int(b)) == (int(ta), int(tc))
    finally:
        pf.pf_tune_clear()
        pf.pf_tune_load(pf.TUNE_TABLE)
