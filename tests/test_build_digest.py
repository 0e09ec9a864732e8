"""The binding never loads a stale library: liblbm.so carries the digest of the
sources it was built from, and load() rebuilds when the tree's sources differ
(CPU; nothing here runs on a GPU)."""
import os
import shutil

from paper_1510_07328_amd import build as B
from paper_1510_07328_amd import lbm


def test_built_library_matches_the_tree():
    # __graft_entry__.build() runs before the tests; the stamp must name these sources
    assert os.path.exists(B.LIB)
    assert B.built_digest() == B.source_digest()
    assert B.is_current()


def test_digest_changes_with_any_source_byte(tmp_path, monkeypatch):
    csrc = tmp_path / "pkg" / "csrc"
    inc = tmp_path / "include"
    shutil.copytree(B.CSRC, csrc)
    shutil.copytree(os.path.join(B.ROOT, "include"), inc)
    monkeypatch.setattr(B, "CSRC", str(csrc))
    monkeypatch.setattr(B, "ROOT", str(tmp_path))
    d0 = B.source_digest()
    assert d0 == B.source_digest()  # deterministic
    f = csrc / "lbm_collide.h"
    f.write_bytes(f.read_bytes() + b" ")
    d1 = B.source_digest()
    assert d1 != d0
    h = inc / "lbm.h"
    h.write_bytes(h.read_bytes().replace(b"LBM_OK = 0", b"LBM_OK  = 0"))
    assert B.source_digest() not in (d0, d1)


def test_load_rebuilds_a_stale_library(monkeypatch):
    calls = []
    monkeypatch.setattr(lbm, "_lib", None)
    monkeypatch.setattr(B, "is_current", lambda: False)
    monkeypatch.setattr(B, "build", lambda *a, **k: calls.append(1) or B.LIB)
    lib = lbm.load()
    assert calls == [1]
    assert hasattr(lib, "lbm_step")
    monkeypatch.setattr(lbm, "_lib", None)
    monkeypatch.setattr(B, "is_current", lambda: True)
    lbm.load()
    assert calls == [1]  # a current library is loaded as it is


def test_oracle_library_carries_its_digest_too():
    from oracle import build as OB
    from oracle import lbm as OL

    OL.lib()
    assert OB.is_current()
