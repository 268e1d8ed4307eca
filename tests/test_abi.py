"""CPU checks of the C-ABI library: it loads, exports every function the
header declares, sizes workspaces and rejects bad parameters (no device call)."""
import ctypes
import os
import re

import pytest

import paper_2308_00763_amd as pf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pf.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(pf_[a-z_]+)\s*\(", src, re.M)))


def test_header_declares_the_binding_names():
    assert _declared() == sorted(pf.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(pf.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name
    assert pf.pf_abi_version() == pf.PF_ABI_VERSION


def test_params_struct_matches_header_size():
    # 4 + 4 + 8 + 6*4 + 8 + 6*8 + 8 + 4 + 4 = 112 bytes on x86-64
    assert ctypes.sizeof(pf.pf_params) == 112


def test_workspace_sizes():
    p64 = pf.make_params(1 << 20, 1024, 1024, "f64")
    p16 = pf.make_params(1 << 20, 1024, 1024, "f16")
    b64, b16 = pf.pf_workspace_bytes(p64), pf.pf_workspace_bytes(p16)
    # state (2 planes) + propagated (2 planes) + prefix (1)
    assert b64 >= (1 << 20) * (4 * 8 + 8)
    assert b16 >= (1 << 20) * (4 * 2 + 4)
    assert b16 < b64 / 2.5
    pd = pf.make_params(1 << 20, 1024, 1024, "f16", diagnostics=True)
    # (a filter with diagnostics resamples at once: compare with the layout
    # without the deferred-resampling buffers)
    assert pf.pf_workspace_bytes(pd) >= pf.pf_member_bytes(p16) + (1 << 20) * 16


@pytest.mark.parametrize("field,value", [
    ("n_particles", 0), ("n_particles", (1 << 28) + 1), ("disk_radius", 0), ("disk_radius", 33),
    ("width", 10), ("dtype", 7), ("fg", 300), ("lik_norm", 5), ("kappa", 0.0),
    ("sigma_x", -1.0), ("x0", float("nan")), ("flags", 8), ("struct_size", 12)])
def test_bad_params_are_rejected(field, value):
    p = pf.make_params(1000, 128, 128)
    setattr(p, field, value)
    with pytest.raises(pf.PfError) as ei:
        pf.pf_workspace_bytes(p)
    assert ei.value.code == pf.PF_ERR_INVALID_ARG
    assert len(pf.pf_last_error()) > 0


def test_null_pointers_are_rejected_without_a_device():
    L = pf.lib()
    p = pf.make_params(1000, 128, 128)
    assert L.pf_workspace_bytes(ctypes.byref(p), None) == pf.PF_ERR_INVALID_ARG
    out = ctypes.c_void_p()
    assert L.pf_init(ctypes.byref(p), None, 0, None, ctypes.byref(out)) == pf.PF_ERR_INVALID_ARG
    assert L.pf_step(None, None, 0) == pf.PF_ERR_INVALID_ARG
    assert L.pf_estimate(None, None) == pf.PF_ERR_INVALID_ARG
    assert L.pf_destroy(None) == pf.PF_OK
    # a workspace pointer that is too small is refused before any device work
    assert L.pf_init(ctypes.byref(p), ctypes.c_void_p(256), 16, None,
                     ctypes.byref(out)) == pf.PF_ERR_WORKSPACE
    assert L.pf_init(ctypes.byref(p), ctypes.c_void_p(257), 1 << 30, None,
                     ctypes.byref(out)) == pf.PF_ERR_INVALID_ARG


def test_batch_workspace_is_the_sum_of_its_filters_plus_the_plan():
    ps = [pf.make_params(n, 256, 256, "f16", stream_id=i) for i, n in enumerate([256, 1000, 5000, 65536])]
    total = pf.pf_batch_workspace_bytes(ps)
    singles = sum(pf.pf_member_bytes(p) for p in ps)
    tiles = sum((p.n_particles + 1023) // 1024 for p in ps)
    # two plans (eager and captured steps): 32 bytes per filter and, per tile,
    # 4 for the tile map and 4 for the pass-A tile list, each
    assert total >= singles + 2 * (8 * tiles + 32 * len(ps))
    assert total < singles + 8192 + 16 * tiles + 450 * len(ps)


def test_member_bytes_leave_out_the_deferred_resampling_buffers():
    # an FP64 or FP32 filter of its own that defers its resampling (at most
    # 2^20 particles, systematic, no diagnostics or variants) holds a second
    # set of propagated positions (2 planes) and prefix sums and an end-slot
    # column; a batch member does not
    for dt, elt, qel in (("f64", 8, 8), ("f32", 4, 4), ("f16", 2, 4), ("bf16", 2, 4)):
        for n in (1, 1000, 1025, 1 << 20):
            pad = -(-n // 1024) * 1024
            tiles = pad // 1024
            p = pf.make_params(n, 1024, 1024, dt)
            extra = 2 * (-(-elt * pad // 256) * 256) + (-(-qel * pad // 256) * 256) + (-(-4 * tiles // 256) * 256)
            if dt in ("f16", "bf16"):  # the 16-bit modes resample at once
                extra = 0
            assert pf.pf_workspace_bytes(p) == pf.pf_member_bytes(p) + extra, (dt, n)
        for p in (pf.make_params((1 << 20) + 1, 1024, 1024, dt), pf.make_params(5000, 1024, 1024, dt, diagnostics=True),
                  pf.make_params(5000, 1024, 1024, dt, metropolis_steps=8), pf.make_params(5000, 1024, 1024, dt, state_only=True)):
            assert pf.pf_workspace_bytes(p) == pf.pf_member_bytes(p)


def test_batch_params_are_checked_per_filter():
    good = pf.make_params(1000, 128, 128, "f16")
    bad = pf.make_params(1000, 128, 128, "f16", radius=0)
    with pytest.raises(pf.PfError) as ei:
        pf.pf_batch_workspace_bytes([good, good, bad])
    assert ei.value.code == pf.PF_ERR_INVALID_ARG and "filter 2" in pf.pf_last_error()
    # one dtype per batch
    with pytest.raises(pf.PfError):
        pf.pf_batch_workspace_bytes([good, pf.make_params(1000, 128, 128, "f32")])
    L = pf.lib()
    out = ctypes.c_size_t()
    arr = (pf.pf_params * 1)(good)
    assert L.pf_batch_workspace_bytes(arr, 0, ctypes.byref(out)) == pf.PF_ERR_INVALID_ARG
    assert L.pf_batch_workspace_bytes(None, 1, ctypes.byref(out)) == pf.PF_ERR_INVALID_ARG
    assert L.pf_batch_workspace_bytes(arr, 1, None) == pf.PF_ERR_INVALID_ARG


def test_batch_null_handles_are_rejected_without_a_device():
    L = pf.lib()
    assert L.pf_batch_step(None, None, None, None) == pf.PF_ERR_INVALID_ARG
    assert L.pf_batch_estimates(None, None) == pf.PF_ERR_INVALID_ARG
    out = ctypes.c_void_p()
    assert L.pf_batch_filter(None, 0, ctypes.byref(out)) == pf.PF_ERR_INVALID_ARG
    assert L.pf_batch_destroy(None) == pf.PF_OK
    good = pf.make_params(1000, 128, 128, "f16")
    arr = (pf.pf_params * 1)(good)
    assert L.pf_batch_init(arr, 1, ctypes.c_void_p(256), 16, None,
                           ctypes.byref(out)) == pf.PF_ERR_WORKSPACE


def test_state_only_workspace_holds_only_the_state():
    # block + two position planes of N_pad elements (tiles of 1024)
    for dt, elt in (("f64", 8), ("f32", 4), ("f16", 2), ("bf16", 2)):
        for n in (1, 1000, 1025, 1 << 20):
            pad = -(-n // 1024) * 1024
            p = pf.make_params(n, 1024, 1024, dt, state_only=True)
            assert pf.pf_workspace_bytes(p) == 256 + 2 * (-(-elt * pad // 256) * 256)
            assert pf.pf_workspace_bytes(p) < pf.pf_workspace_bytes(pf.make_params(n, 1024, 1024, dt)) / 2
    src = open(HEADER).read()
    assert "#define PF_STATIC_SCRATCH_BYTES (24u * 1024u * 1024u + 64u * 1024u)" in src
    assert pf.PF_STATIC_SCRATCH_BYTES == 24 * 1024 * 1024 + 64 * 1024


@pytest.mark.parametrize("dt,n_ok,n_bad", [("f64", 1 << 20, (1 << 20) + 1),
                                           ("f32", (1 << 21) - 5 * 1024, 1 << 21),
                                           ("f16", 3_100_000, 3_200_000)])
def test_state_only_size_limit(dt, n_ok, n_bad):
    pf.pf_workspace_bytes(pf.make_params(n_ok, 1024, 1024, dt, state_only=True))
    with pytest.raises(pf.PfError) as ei:
        pf.pf_workspace_bytes(pf.make_params(n_bad, 1024, 1024, dt, state_only=True))
    assert ei.value.code == pf.PF_ERR_INVALID_ARG and "static scratch" in pf.pf_last_error()


@pytest.mark.parametrize("variant", [dict(naive_likelihood=True), dict(naive_resample=True),
                                     dict(metropolis_steps=8), dict(gumbel_max=True),
                                     dict(rejection_trials=64)])
def test_state_only_takes_only_the_default_step(variant):
    with pytest.raises(pf.PfError) as ei:
        pf.pf_workspace_bytes(pf.make_params(1000, 128, 128, "f16", state_only=True, **variant))
    assert ei.value.code == pf.PF_ERR_INVALID_ARG


def test_state_only_filters_are_not_batched():
    ps = [pf.make_params(1000, 128, 128, "f16", state_only=True)]
    with pytest.raises(pf.PfError):
        pf.pf_batch_workspace_bytes(ps)


def test_rejection_trials_field():
    # rejection resampling keeps at most 64 v trials per slot (v in the
    # shared field), and excludes every other resampler
    p = pf.make_params(1000, 128, 128, rejection_trials=640)
    assert p.flags & pf.PF_FLAG_REJECTION
    assert (p.flags >> pf.PF_METROPOLIS_STEPS_SHIFT) & 0xFF == 10
    with pytest.raises(ValueError):
        pf.make_params(1000, 128, 128, rejection_trials=100)
    with pytest.raises(pf.PfError):
        pf.pf_workspace_bytes(pf.make_params(1000, 128, 128, rejection_trials=64, metropolis_steps=8))
