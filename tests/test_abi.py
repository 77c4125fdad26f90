"""The C ABI: exported symbols (CPU) and error / per-pair status behaviour (GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT


def header_functions():
    src = open(os.path.join(ROOT, "include", "gk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gk_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_expected_api():
    fns = header_functions()
    for name in ("gk_create", "gk_destroy", "gk_last_error", "gk_load_reference",
                 "gk_encode_reads", "gk_filter"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    from paper_2103_14978_amd import gk
    lib = ctypes.CDLL(gk.LIB_PATH)
    for name in header_functions():
        assert hasattr(lib, name), f"{name} declared in gk.h but not exported"
    assert set(gk.EXPORTED) <= set(header_functions())


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2103_14978_amd import gk
    monkeypatch.setattr(gk, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gk, "_lib", None)
    with pytest.raises(ImportError):
        gk.lib()


def test_create_rejects_null_out():
    from paper_2103_14978_amd import gk
    L = gk.lib()
    assert L.gk_create(0, None) == gk.GK_EINVAL
    assert "NULL" in gk.gk_last_error(None)


# ------------------------------------------------------------------ GPU ---

@pytest.mark.gpu
def test_errors(gkctx):
    import torch
    from paper_2103_14978_amd import device, gk
    ctx2 = gk.gk_create(0)
    try:
        reads = device.encode_reads(ctx2, np.frombuffer(b"ACGT", np.uint8),
                                    np.array([0, 4], np.uint64))
        pairs = device.upload_pairs(np.array([0], np.uint32), np.array([0], np.uint32))
        b = device.batch_for(reads, pairs, e_uniform=0)
        with pytest.raises(gk.GkError) as ei:
            gk.gk_filter(ctx2, b)                       # no reference yet
        assert ei.value.status == gk.GK_ENOREF
        gk.gk_load_reference(ctx2, b"ACGTACGT")
        assert gk.gk_reference_info(ctx2) == (8, 0)
        for field, value in (("max_read_len", 0), ("max_read_len", 513), ("e_uniform", 256),
                             ("pitch", 0)):
            bad = device.batch_for(reads, pairs, e_uniform=0)
            setattr(bad, field, value)
            if field == "pitch":
                bad.n_reads = 1
            with pytest.raises(gk.GkError) as ei:
                gk.gk_filter(ctx2, bad)
            assert ei.value.status == gk.GK_EINVAL, field
        bad = device.batch_for(reads, pairs, e_uniform=0)
        bad.accept = None
        with pytest.raises(gk.GkError) as ei:
            gk.gk_filter(ctx2, bad)
        assert ei.value.status == gk.GK_EINVAL
        bad = device.batch_for(reads, pairs, e_uniform=0)
        bad.n_pairs = 1 << 38
        with pytest.raises(gk.GkError) as ei:
            gk.gk_filter(ctx2, bad)
        assert ei.value.status == gk.GK_ERANGE
        # empty batch is fine
        ok = device.batch_for(reads, pairs, e_uniform=0)
        ok.n_pairs = 0
        gk.gk_filter(ctx2, ok)
        with pytest.raises(gk.GkError) as ei:
            gk.gk_load_reference(ctx2, b"")
        assert ei.value.status == gk.GK_EINVAL
        bad = device.batch_for(reads, pairs, e_uniform=0)
        bad.read_layout = 7
        with pytest.raises(gk.GkError) as ei:
            gk.gk_filter(ctx2, bad)
        assert ei.value.status == gk.GK_EINVAL
        for opt, val in ((gk.GK_OPT_PAIRS_PER_LANE, -1), (gk.GK_OPT_PAIRS_PER_LANE, 65537),
                         (gk.GK_OPT_HOST_ENCODE_THREADS, -1),
                         (gk.GK_OPT_HOST_ENCODE_THREADS, 65),
                         (gk.GK_OPT_HOST_CHUNK_PAIRS, 63),
                         (gk.GK_OPT_HOST_CHUNK_PAIRS, (1 << 26) + 1),
                         (gk.GK_OPT_SERVER_COPY_STREAMS, 0),
                         (gk.GK_OPT_SERVER_COPY_STREAMS, 9), (999, 0)):
            with pytest.raises(gk.GkError) as ei:
                gk.gk_set_option(ctx2, opt, val)
            assert ei.value.status == gk.GK_EINVAL
        gk.gk_set_option(ctx2, gk.GK_OPT_PAIRS_PER_LANE, 5)
        assert gk.gk_get_option(ctx2, gk.GK_OPT_PAIRS_PER_LANE) == 5
        assert gk.gk_get_option(ctx2, gk.GK_OPT_HOST_ENCODE_THREADS) == 0
        gk.gk_set_option(ctx2, gk.GK_OPT_HOST_ENCODE_THREADS, 64)
        assert gk.gk_get_option(ctx2, gk.GK_OPT_HOST_ENCODE_THREADS) == 64
        assert gk.gk_get_option(ctx2, gk.GK_OPT_HOST_CHUNK_PAIRS) == 0
        gk.gk_set_option(ctx2, gk.GK_OPT_HOST_CHUNK_PAIRS, 1 << 26)
        assert gk.gk_get_option(ctx2, gk.GK_OPT_HOST_CHUNK_PAIRS) == 1 << 26
        assert gk.gk_get_option(ctx2, gk.GK_OPT_SERVER_COPY_STREAMS) == 4
        gk.gk_set_option(ctx2, gk.GK_OPT_SERVER_COPY_STREAMS, 1)
        assert gk.gk_get_option(ctx2, gk.GK_OPT_SERVER_COPY_STREAMS) == 1
        torch.cuda.synchronize()
    finally:
        gk.gk_destroy(ctx2)


@pytest.mark.gpu
def test_per_pair_status(gkctx):
    """Unknown bases (read or window), windows past the end, lowercase,
    invalid lengths and read indices, against the oracle."""
    from gpu_cases import concat_reads, run_gpu, run_oracle, assert_same, say
    import oracle
    rng = np.random.default_rng(5)
    ref = bytearray(rng.choice(np.frombuffer(b"ACGT", np.uint8), 5000).tobytes())
    for p in (100, 101, 102, 700, 2047, 2048, 4000):
        ref[p] = ord("N")
    ref[3000:3010] = b"acgtacgtnn"
    ref = np.frombuffer(bytes(ref), np.uint8).copy()
    seqs = [ref[10:110].tobytes(), ref[50:150].tobytes(), b"ACGTNACGTA" * 10,
            ref[2990:3090].tobytes(), ref[4900:5000].tobytes(), b"", b"A" * 600,
            ref[0:64].tobytes().lower(), b"acgtXacgt" + b"A" * 91]
    reads, off = concat_reads(seqs)
    pr = np.array([0, 1, 1, 2, 3, 4, 4, 4, 5, 6, 7, 8, 0, 0], np.uint32)
    pos = np.array([10, 50, 60, 200, 2990, 4900, 4901, 5000, 0, 0, 0, 300, 4950, 0xFFFFFFF0],
                   np.uint32)
    say("case: per-pair status")
    a, s, _ = run_gpu(gkctx, ref, reads, off, pr, pos, 3, max_read_len=512)
    ra, rs = run_oracle(ref, reads, off, pr, pos, 3)
    assert_same(a, s, ra, rs, "status")
    assert a[3] == oracle.UNDEFINED and a[6] == oracle.UNDEFINED and a[7] == oracle.UNDEFINED
    assert a[8] == oracle.INVALID and a[9] == oracle.INVALID and a[13] == oracle.UNDEFINED
    # read index out of range -> INVALID
    pr2 = np.array([7, 9, 1000], np.uint32)          # read 7: lower-case copy of ref[0:64]
    pos2 = np.array([0, 10, 10], np.uint32)
    a2, s2, _ = run_gpu(gkctx, ref, reads, off, pr2, pos2, 3, max_read_len=512, load_ref=False)
    assert list(a2) == [oracle.ACCEPT, oracle.INVALID, oracle.INVALID]
    assert list(s2[1:]) == [oracle.EST_NONE, oracle.EST_NONE]
    # a read longer than max_read_len -> INVALID
    a3, s3, _ = run_gpu(gkctx, ref, reads, off, np.array([4], np.uint32),
                        np.array([4900], np.uint32), 3, max_read_len=64, load_ref=False)
    assert a3[0] == oracle.INVALID


@pytest.mark.gpu
@pytest.mark.parametrize("layout", [0, 1], ids=["split", "interleaved"])
def test_encode_reads_layout(gkctx, layout):
    """gk_encode_reads against an independent packing of the documented
    layouts: base i of a read in word i / 16 (word w of read r at
    w * pitch + r), A=0 C=1 G=2 T=3; split: low code bit at bit i mod 16, high
    bit at 16 + i mod 16; interleaved: code at bits 2(i mod 16), 2(i mod 16)+1."""
    from paper_2103_14978_amd import device
    rng = np.random.default_rng(9)
    seqs = []
    for i in range(300):
        m = int(rng.integers(0, 200))
        s = bytearray(rng.choice(np.frombuffer(b"ACGTacgt", np.uint8), m).tobytes())
        if i % 17 == 0 and m:
            s[int(rng.integers(0, m))] = ord("N")
        seqs.append(bytes(s))
    from gpu_cases import concat_reads
    reads, off = concat_reads(seqs)
    dr = device.encode_reads(gkctx, reads, off, max_len=200, layout=layout)
    packed = dr.packed.cpu().numpy().view(np.uint32).reshape(-1, dr.pitch)
    lens = dr.read_len.cpu().numpy().view(np.uint16)[:len(seqs)]
    hasn = dr.has_n.cpu().numpy()[:len(seqs)]
    code = {ord(c): v for c, v in zip("ACGTacgt", [0, 1, 2, 3, 0, 1, 2, 3])}
    for r, s in enumerate(seqs):
        assert lens[r] == len(s)
        assert hasn[r] == int(any(ch not in code for ch in s))
        want = [0] * packed.shape[0]
        for i, ch in enumerate(s):
            c = code.get(ch, 0)
            if layout == 0:
                want[i // 16] |= ((c & 1) << (i % 16)) | ((c >> 1) << (16 + i % 16))
            else:
                want[i // 16] |= c << (2 * (i % 16))
        assert [int(x) for x in packed[:, r]] == want, r


@pytest.mark.gpu
def test_tiny_and_odd_references(gkctx):
    """References of every small length load (chunking must always advance)
    and filter against the oracle, including reads that end exactly at the
    reference end."""
    from gpu_cases import concat_reads, run_gpu, run_oracle, assert_same, say
    from paper_2103_14978_amd import gk
    rng = np.random.default_rng(21)
    for L in (1, 2, 7, 31, 32, 33, 63, 64, 65, 95, 96, 97, 1000):
        ref = rng.choice(np.frombuffer(b"ACGT", np.uint8), L).copy()
        say(f"case: tiny reference L={L}")
        gk.gk_load_reference(gkctx, ref)
        assert gk.gk_reference_info(gkctx) == (L, 0)
        seqs = [ref[max(0, L - m):L].tobytes() for m in (1, 2, 5, 17, 40) if m <= L]
        seqs += [ref[:min(L, 33)].tobytes()]
        reads, off = concat_reads(seqs)
        pr = np.arange(len(seqs), dtype=np.uint32)
        pos = np.array([max(0, L - len(s)) for s in seqs[:-1]] + [0], np.uint32)
        for e in (0, 1, 3):
            a, s, _ = run_gpu(gkctx, ref, reads, off, pr, pos, e, max_read_len=64, load_ref=False)
            ra, rs = run_oracle(ref, reads, off, pr, pos, e)
            assert_same(a, s, ra, rs, f"tiny L={L} e={e}")


@pytest.mark.gpu
def test_options_from_environment(monkeypatch):
    """gk_create takes GK_<name> for each option GK_OPT_<name>; a value that is
    not an integer in range fails the call with GK_EINVAL, naming the
    variable, and later contexts without it are unaffected."""
    from paper_2103_14978_amd import gk
    monkeypatch.setenv("GK_MIXED_TILE", "8192")
    monkeypatch.setenv("GK_HOST_CHUNK_PAIRS", "65536")
    monkeypatch.setenv("GK_SERVER_PART_PAIRS", "4096")
    ctx = gk.gk_create(0)
    try:
        assert gk.gk_get_option(ctx, gk.GK_OPT_MIXED_TILE) == 8192
        assert gk.gk_get_option(ctx, gk.GK_OPT_HOST_CHUNK_PAIRS) == 65536
        assert gk.gk_get_option(ctx, gk.GK_OPT_SERVER_PART_PAIRS) == 4096
        assert gk.gk_get_option(ctx, gk.GK_OPT_MIXED_GRAPH) == 1
    finally:
        gk.gk_destroy(ctx)
    for var, val in (("GK_MIXED_TILE", "3000"), ("GK_MIXED_TILE", "4k"),
                     ("GK_HOST_ENCODE_THREADS", ""), ("GK_PAIRS_PER_LANE", "-1")):
        monkeypatch.setenv(var, val)
        with pytest.raises(gk.GkError) as ei:
            gk.gk_create(0)
        assert ei.value.status == gk.GK_EINVAL
        assert var in str(ei.value)
        monkeypatch.delenv(var)
    monkeypatch.delenv("GK_HOST_CHUNK_PAIRS")
    monkeypatch.delenv("GK_SERVER_PART_PAIRS")
    ctx = gk.gk_create(0)
    try:
        assert gk.gk_get_option(ctx, gk.GK_OPT_MIXED_TILE) == 4096
        assert gk.gk_get_option(ctx, gk.GK_OPT_HOST_CHUNK_PAIRS) == 0
    finally:
        gk.gk_destroy(ctx)


@pytest.mark.gpu
def test_fault_injection_from_environment(monkeypatch):
    """GK_FAULT_INJECT=alloc:N arms the allocation failure once per process:
    with N = 1 the first gk_create's own allocation fails (GK_ENOMEM) and the
    next gk_create works; a malformed value fails gk_create with GK_EINVAL."""
    from paper_2103_14978_amd import gk
    for val in ("alloc:0", "alloc:-3", "alloc", "memory:2", "alloc:2x"):
        monkeypatch.setenv("GK_FAULT_INJECT", val)
        with pytest.raises(gk.GkError) as ei:
            gk.gk_create(0)
        assert ei.value.status == gk.GK_EINVAL and "GK_FAULT_INJECT" in str(ei.value)
    monkeypatch.setenv("GK_FAULT_INJECT", "alloc:1")
    with pytest.raises(gk.GkError) as ei:
        gk.gk_create(0)
    assert ei.value.status == gk.GK_ENOMEM
    ctx = gk.gk_create(0)           # armed once: this one allocates normally
    gk.gk_destroy(ctx)
    monkeypatch.delenv("GK_FAULT_INJECT")
