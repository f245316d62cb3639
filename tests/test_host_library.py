"""Host-side parts of the library, on the CPU: the ABI exports every declared symbol,
the builder's BWT (SA-IS) equals the oracle's direct-comparison BWT, and the 2-bit
packing follows Fig. 2. No GPU call is made."""
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_1811_06127_amd import fm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")
CODE = {"a": 0, "c": 1, "g": 2, "t": 3}


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fm_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import subprocess
    names = declared_functions()
    assert len(names) >= 20
    out = subprocess.check_output(["nm", "-D", "--defined-only", fm.LIB_PATH], text=True)
    exported = set(re.findall(r" T (fm_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = fm.lib()
    for n in names:
        getattr(lib, n)


def test_header_is_plain_c(tmp_path):
    """include/fm.h compiles as C99 and as C++17 with warnings as errors: the boundary
    holds plain types only."""
    import shutil
    import subprocess
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = tmp_path / "use_fm.c"
    src.write_text('#include "fm.h"\nint main(void) { fm_tuning t; t.order = 1; return (int)t.order + FM_OP_LOCATE; }\n')
    for cc, std, lang in (("gcc", "-std=c99", "c"), ("g++", "-std=c++17", "c++")):
        if shutil.which(cc) is None:
            pytest.skip("no %s" % cc)
        subprocess.run([cc, std, "-Wall", "-Wextra", "-Werror", "-fsyntax-only", "-I", inc, "-x", lang, str(src)],
                       check=True)


def test_strerror_and_version():
    assert fm.strerror(fm.FM_OK) == "ok"
    assert fm.strerror(fm.FM_EOVERFLOW) == "hit capacity exceeded"
    assert fm.lib().fm_version() == 1


def read_golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split(None, 1)
            out[k] = v
    return out


def test_fig2_packing_word_and_counts():
    g = read_golden("fig2_word.txt")
    s = g["STRING"]
    codes = np.array([CODE[c] for c in s], np.uint8)
    words = fm.fm_pack_host(codes)
    assert words.size == 2
    word = int(words[0]) | (int(words[1]) << 32)
    assert word == int(g["WORD"], 16)
    assert word & 0x0F0F0F0F0F0F0F0F == int(g["LOW_NIBBLES"], 16)
    assert (word >> 4) & 0x0F0F0F0F0F0F0F0F == int(g["HIGH_NIBBLES"], 16)
    # decoding the word two bits at a time, least significant first, gives back the string
    dec = [(word >> (2 * j)) & 3 for j in range(32)]
    assert dec == codes.tolist()
    assert dec.count(CODE["g"]) == int(g["COUNT_G"])


def test_pack_rejects_non_bases():
    with pytest.raises(fm.FmError):
        fm.fm_pack_host(np.array([0, 1, 4], np.uint8))


@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (17, 3), (1000, 4), (65536, 5)])
def test_builder_bwt_equals_oracle(n, seed):
    R = synth.iid_reference(n, seed)
    bwt, dr = fm.fm_bwt_host(R)
    x = oracle.OracleIndex(R)
    assert dr == x.dollar_row
    assert np.array_equal(bwt, x.bwt)


def test_builder_bwt_equals_oracle_repetitive():
    # repeats and runs stress the induced sorting's recursion
    R = synth.reference_with_repeats(120_000, 9, copy_frac=0.2, copy_len=(500, 5000), copy_sub=0.0,
                                     tandem_frac=0.1, tandem_unit=(1, 7), tandem_len=(100, 3000))
    bwt, dr = fm.fm_bwt_host(R)
    x = oracle.OracleIndex(R)
    assert dr == x.dollar_row
    assert np.array_equal(bwt, x.bwt)
    for R in (np.zeros(500, np.uint8), np.tile(np.array([0, 1], np.uint8), 300)):
        bwt, dr = fm.fm_bwt_host(R)
        x = oracle.OracleIndex(R)
        assert dr == x.dollar_row and np.array_equal(bwt, x.bwt)


def test_builder_rejects_bad_codes():
    with pytest.raises(fm.FmError):
        fm.fm_bwt_host(np.array([0, 5, 1], np.uint8))


def test_index_file_roundtrip_header(tmp_path):
    R = synth.iid_reference(5000, 12)
    p = str(tmp_path / "x.fmi")
    fm.fm_index_build_file(R, p, fm.FM_LOAD_REVERSE)
    raw = open(p, "rb").read()
    assert raw[:8] == b"FMOCC001"
    hdr = np.frombuffer(raw[8:8 + 8 * 16], np.uint64)
    x = oracle.OracleIndex(R)
    assert hdr[0] == 5000 and hdr[2] == x.dollar_row
    assert hdr[3:8].tolist() == x.C.tolist()
    words = int(hdr[14])
    assert words == (5001 + 15) // 16
    assert len(raw) == 8 + 8 * 16 + 2 * 4 * words
