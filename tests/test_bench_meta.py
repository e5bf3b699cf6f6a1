"""The benchmark's bookkeeping, on the CPU: the kernel hash that ties stored
counter results (profiles/) to the kernels they were taken from, and the
algorithmic byte model of the CG iteration's passes."""

import os
import shutil

import bench
from paper_1305_3625_amd import build


def _copy_sources(tmp, edit=None):
    for p in bench.KERNEL_SOURCES:
        dst = os.path.join(tmp, p)
        os.makedirs(os.path.dirname(dst), exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, p), dst)
    if edit:
        p, fn = edit
        path = os.path.join(tmp, p)
        with open(path) as f:
            s = f.read()
        with open(path, "w") as f:
            f.write(fn(s))


def test_kernel_hash_ignores_comments_and_checkout_path(tmp_path, monkeypatch):
    h0 = bench.kernel_hash()
    src = bench.KERNEL_SOURCES[0]
    _copy_sources(str(tmp_path), (src, lambda s: "// a comment line\n" + s.replace("\n", "\n  ", 3)))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_hash() == h0
    # the include directories name the checkout, which differs between machines
    flags = [f if not f.startswith("-I") else "-I/elsewhere" + f[2:] for f in build.CXXFLAGS]
    monkeypatch.setattr(build, "CXXFLAGS", flags)
    assert bench.kernel_hash() == h0


def test_kernel_hash_follows_code_and_flags(tmp_path, monkeypatch):
    h0 = bench.kernel_hash()
    src = bench.KERNEL_SOURCES[0]
    _copy_sources(str(tmp_path), (src, lambda s: s + "\nnamespace { constexpr int kExtra = 1; }\n"))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_hash() != h0
    monkeypatch.undo()
    monkeypatch.setattr(build, "CXXFLAGS", build.CXXFLAGS + ["-DFFTCG_SOMETHING=1"])
    assert bench.kernel_hash() != h0


def test_byte_model_of_the_iteration():
    """Per pass at L = 2048 (M = 4096, N = 2048 packed columns): the folded
    iteration moves 8 L^2 bytes less than the separate one (q is neither
    written nor read; r is read and written by the row-inverse pass), and
    the turn pass 8 L^2 less again."""
    L, M = 2048, 4096
    bm = bench.bytes_model(L, M)
    n, W = L * L, 8 * L * (M // 2)
    ps = bm["passes"]
    assert ps["row_fwd"] == 20 * n + W
    assert ps["row_inv"] == W + 12 * n and ps["row_inv_upd"] == W + 16 * n and ps["update"] == 12 * n
    assert bm["iteration"] == ps["row_fwd"] + ps["col"] + ps["row_inv"] + ps["update"]
    assert bm["iteration_folded"] == ps["row_fwd"] + ps["col"] + ps["row_inv_upd"]
    assert bm["iteration"] - bm["iteration_folded"] == 8 * n
    assert round(bm["iteration_folded"] / 1e6, 1) == 302.0
    # the turn pass: row_inv_upd then row_fwd on the same rows, without
    # reading back r (written by the first half) and p (held from it)
    assert ps["turn"] == ps["row_inv_upd"] + ps["row_fwd"] - 8 * n
    assert bm["iteration_turn"] == ps["col"] + ps["turn"] == bm["iteration_folded"] - 8 * n
    names = bench.pass_kernels(M)
    assert set(names) == set(ps)
