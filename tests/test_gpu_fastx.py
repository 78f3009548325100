"""FASTQ / FASTA text through the front end and the HIP path: the countBF
words, distinct, trustworthy and erroneous lists and the window count equal
the oracle's on the same parsed reads, one read per record and in
one-sequence mode (windows across record boundaries)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2305_07545_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    P.load_library()


def fastq_text(rs, width=60):
    out = []
    for i in range(rs.n_reads):
        s = bytes(rs.reads[int(rs.offsets[i]):int(rs.offsets[i + 1])])
        out.append(b"@r%d\n" % i + b"\n".join(s[j:j + width] for j in range(0, len(s), width))
                   + b"\n+\n" + b"I" * len(s) + b"\n")
    return b"".join(out)


@pytest.mark.parametrize("one_sequence", [False, True])
def test_fastq_front_end_matches_oracle(one_sequence):
    rs = synth.random_reads(611, 3000, 20, 300, k=21, tau=2, p_n=0.01)
    text = fastq_text(rs)
    reads, offs = P.parse_fastx(text, one_sequence=one_sequence)
    if not one_sequence:
        assert np.array_equal(reads, rs.reads) and np.array_equal(offs, rs.offsets)
    X, Y = oracle.dims(2 * rs.n_items)
    print(f"case fastx one_sequence={one_sequence}: bases={len(reads)} reads={len(offs) - 1}",
          flush=True)
    g = P.run_kmerco(torch.from_numpy(reads).cuda(),
                     torch.from_numpy(offs.view(np.int64)).cuda(), 21, 2, X, Y)
    c = oracle.run_kmerco(reads, offs, 21, 2, X, Y)
    for a, b in zip(g[:4], c[:4]):
        assert np.array_equal(np.asarray(a, dtype=np.uint64), np.asarray(b, dtype=np.uint64))
    assert g[4] == c[4]
