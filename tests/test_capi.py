"""The C-ABI library loads and exports every symbol include/he.h declares (no GPU).

Also checks the host-only prime helper against the oracle's prime rule.
"""
import os
import re

import pytest

from oracle import params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "he.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(he_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2104_09164_amd import he
    if not os.path.exists(he.LIB_PATH):
        pytest.fail("libhe.so is not built: run __graft_entry__.build()")
    return he.lib()


def test_exports_every_declared_symbol(lib):
    from paper_2104_09164_amd import he
    syms = declared_symbols()
    assert len(syms) >= 25
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing
    assert set(syms) == set(he.EXPORTED)


def test_strerror(lib):
    assert lib.he_strerror(0) == b"ok"
    assert b"key" in lib.he_strerror(-3)


@pytest.mark.parametrize("name", ["cfg1", "cfg3", "cfg4"])
def test_gen_primes_matches_oracle_rule(lib, name):
    from paper_2104_09164_amd import he
    pr = params.preset(name)
    qb = [q.bit_length() for q in pr.q]
    pb = [p.bit_length() for p in pr.p]
    q, p = he.prime_chain(pr.log_n, qb, pb)
    assert q == pr.q and p == pr.p


def test_product_path_has_no_oracle_import():
    pkg = os.path.join(ROOT, "paper_2104_09164_amd")
    pat = re.compile(r"(^\s*import\s+oracle|^\s*from\s+oracle|oracle/|liboracle)", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                assert not pat.search(open(os.path.join(dirpath, f)).read()), f


def test_single_hip_runtime_whatever_the_import_order():
    import subprocess
    import sys
    code = ("import os; from paper_2104_09164_amd import he; he.lib(); import torch; "
            "m = open(f'/proc/{os.getpid()}/maps').read(); "
            "print(len({l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, check=True)
    assert out.stdout.strip() == "1"
