"""The FASTA/FASTQ front end (kc_parse_fastx, host code of the library):
records parsed by the library equal the records a plain reference parser in
this file reads, for generated files with random line wrapping, CRLF line
ends, comments, blank lines, empty records and qualities that start with
'@'; sizing and error behaviour of the C call; and the paper's counting
convention in one-sequence mode (a data set of total length L gives
L - K + 1 windows)."""
import ctypes
import os

import numpy as np
import pytest

import oracle

P = pytest.importorskip("paper_2305_07545_amd")


def ref_records(text: bytes):
    """Plain reading of FASTA / FASTQ text: the list of record sequences."""
    lines = [ln[:-1] if ln.endswith(b"\r") else ln for ln in text.split(b"\n")]
    recs = []
    i = 0
    while i < len(lines) and (not lines[i] or lines[i].startswith(b";")):
        i += 1
    if i == len(lines):
        return recs
    if lines[i].startswith(b">"):
        for ln in lines[i:]:
            if not ln or ln.startswith(b";"):
                continue
            if ln.startswith(b">"):
                recs.append(b"")
            else:
                recs[-1] += ln
        return recs
    while i < len(lines):
        if not lines[i]:
            i += 1
            continue
        assert lines[i].startswith(b"@")
        i += 1
        seq = b""
        while not lines[i].startswith(b"+"):
            seq += lines[i]
            i += 1
        i += 1
        q = 0
        while q < len(seq):
            q += len(lines[i])
            i += 1
        recs.append(seq)
    return recs


def render(recs, fastq: bool, rng, crlf: bool):
    nl = b"\r\n" if crlf else b"\n"
    out = []
    if not fastq:
        out.append(b";a comment line")
    for r, seq in enumerate(recs):
        if rng.random() < 0.2:
            out.append(b"")
        width = int(rng.integers(1, 80))
        chunks = [seq[i:i + width] for i in range(0, len(seq), width)] or ([] if not fastq else [b""])
        if fastq:
            out.append(b"@read%d extra" % r)
            out += chunks
            out.append(b"+" if rng.random() < 0.5 else b"+read%d" % r)
            qual = rng.choice(list(b"@I#5+"), size=len(seq)).astype(np.uint8).tobytes()
            qw = int(rng.integers(1, 80))
            out += [qual[i:i + qw] for i in range(0, len(qual), qw)] or [b""]
        else:
            out.append(b">read%d some description" % r)
            out += chunks
    return nl.join(out) + (nl if rng.random() < 0.7 else b"")


def random_records(rng, n):
    return [rng.choice(list(b"ACGTNacgtRY"), p=[.2, .2, .2, .2, .04, .03, .03, .03, .03, .02, .02],
                       size=int(rng.integers(0, 400))).astype(np.uint8).tobytes()
            for _ in range(n)]


@pytest.mark.parametrize("fastq", [False, True])
@pytest.mark.parametrize("crlf", [False, True])
def test_generated_files_match_reference(fastq, crlf):
    rng = np.random.default_rng(90 + 2 * fastq + crlf)
    for trial in range(20):
        recs = random_records(rng, int(rng.integers(0, 30)))
        text = render(recs, fastq, rng, crlf)
        assert ref_records(text) == recs  # the renderer and the reference agree
        seq, offs = P.parse_fastx(text)
        got = [bytes(seq[int(offs[i]):int(offs[i + 1])]) for i in range(len(offs) - 1)]
        assert got == recs, (trial, text[:200])
        one, o1 = P.parse_fastx(text, one_sequence=True)
        assert bytes(one) == b"".join(recs)
        assert list(o1) == ([0, len(one)] if recs else [0])


def test_sizing_and_errors():
    lib = P.load_library()
    text = b">a\nACGT\n>b\nGG\n"
    nb, nr = ctypes.c_uint64(), ctypes.c_uint64()
    seq = (ctypes.c_uint8 * 16)(*([7] * 16))
    off = (ctypes.c_uint64 * 8)(*([9] * 8))
    # too small: counts report the need, nothing beyond the capacities is written
    st = lib.kc_parse_fastx(text, len(text), 0, seq, 3, off, 2, ctypes.byref(nb), ctypes.byref(nr))
    assert st == P.kmerco.KC_ERANGE and (nb.value, nr.value) == (6, 2)
    assert bytes(seq[:3]) == b"ACG" and list(seq[3:]) == [7] * 13
    assert list(off[:2]) == [0, 4] and list(off[2:]) == [9] * 6
    st = lib.kc_parse_fastx(text, len(text), 0, seq, 6, off, 3, ctypes.byref(nb), ctypes.byref(nr))
    assert st == 0 and bytes(seq[:6]) == b"ACGTGG" and list(off[:3]) == [0, 4, 6]
    for bad in [b"ACGT\n", b"@r\nACGT\n", b"@r\nACGT\n+\nII\n", b"@r\nAC\n+\nII\nxyz\n",
                b"@r\nAC\n+\nIIII\n"]:
        st = lib.kc_parse_fastx(bad, len(bad), 0, seq, 16, off, 8, ctypes.byref(nb),
                                ctypes.byref(nr))
        assert st == P.kmerco.KC_EINVAL, bad
    assert lib.kc_parse_fastx(text, len(text), 2, seq, 16, off, 8, ctypes.byref(nb),
                              ctypes.byref(nr)) == P.kmerco.KC_EINVAL  # unknown flag
    assert lib.kc_parse_fastx(None, 0, 0, None, 0, off, 1, ctypes.byref(nb),
                              ctypes.byref(nr)) == 0 and (nb.value, nr.value) == (0, 0)
    s, o = P.parse_fastx(b"\n\n")
    assert s.size == 0 and list(o) == [0]


def test_read_fastx_file(tmp_path):
    p = tmp_path / "x.fq"
    p.write_bytes(b"@a\nACGTAC\n+\n@@@@@@\n@b\nTT\n+\n##\n")
    seq, offs = P.read_fastx(str(p))
    assert bytes(seq) == b"ACGTACTT" and list(offs) == [0, 6, 8]
    (tmp_path / "e.fa").write_bytes(b"")
    seq, offs = P.read_fastx(str(tmp_path / "e.fa"))
    assert seq.size == 0 and list(offs) == [0]


def test_one_sequence_counts_L_minus_K_plus_1():
    """The paper's totals (its 28-mer and 55-mer counts differ by 27 for every
    data set) imply one sequence per data set: L - K + 1 windows.  A clean
    multi-record FASTA in one-sequence mode gives exactly that for every K;
    per record it gives the sum of the records' L_r - K + 1."""
    rng = np.random.default_rng(95)
    recs = [rng.choice(list(b"ACGT"), size=int(rng.integers(40, 300))).astype(np.uint8).tobytes()
            for _ in range(12)]
    text = b"".join(b">r\n" + r[:31] + b"\n" + r[31:] + b"\n" for r in recs)
    oracle.build(force=False)
    one, o1 = P.parse_fastx(text, one_sequence=True)
    per, op = P.parse_fastx(text)
    L = len(one)
    for k in (21, 28, 31):
        X, Y = oracle.dims(4 * L)
        nw1 = oracle.run_kmerco(one, o1, k, 2, X, Y)[4]
        nwp = oracle.run_kmerco(per, op, k, 2, X, Y)[4]
        assert nw1 == L - k + 1
        assert nwp == sum(len(r) - k + 1 for r in recs)
