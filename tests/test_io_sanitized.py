"""The file readers (H.DAT, sizeH.dat / sizeBP.dat) under the address and
undefined-behaviour sanitizers: rm_io.cpp is host code, built here with g++
beside a small driver (io_reader_harness.cpp) and run over valid files and over
damaged ones (every truncation, seeded byte flips, extreme counts, broken
record markers, damaged text), and the OMEGA writer over its edge arguments.
A damaged file must end in an error status; any read or write outside a buffer
aborts the sanitized run."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import _fortran as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1909_07321_amd", "csrc", "rm_io.cpp")
HARNESS = os.path.join(ROOT, "tests", "io_reader_harness.cpp")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = tmp_path_factory.mktemp("asan") / "io_reader_harness"
    # the sanitizer runtimes are linked in, so the driver runs under any environment as it is
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-static-libasan",
                           "-static-libubsan", "-I", os.path.join(ROOT, "include"), SRC, HARNESS, "-o", str(exe)],
                          timeout=300)
    return exe


def _run(exe, kind, paths):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:allocator_may_return_null=1:"
                                        "verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe), kind] + [str(p) for p in paths], capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, f"sanitizer report:\n{r.stderr[-4000:]}"
    return r.stdout.splitlines()


def _hdat(big=False, split=0, lamax=2):
    rng = np.random.default_rng(11)
    nast = 3
    enat = np.concatenate([[-1.25], np.sort(rng.uniform(-1.2, 0.5, nast - 1))])
    data = F.hdat_target(10, 14, 2, lamax, enat, np.arange(nast) % 3, np.full(nast, 2), 11.5, 0.0,
                         rng.normal(size=(2, 3)), [(rng.normal(size=2), rng.normal(size=2))] * 2, big)
    for seed, nconat, M in ((1, [2, 0, 3], 7), (2, [1, 2, 1], 5)):
        n = sum(nconat)
        cf = rng.normal(size=(lamax, n, n))
        data += F.hdat_symmetry(3, 2, 1, nconat, rng.integers(0, 6, n), cf + np.transpose(cf, (0, 2, 1)),
                                np.sort(rng.uniform(-2, 40, M)), rng.normal(size=(M, n)), big=big, split=split)
    return data


def test_hdat_reader_under_sanitizers(harness, tmp_path):
    files, valid = [], []

    def put(name, data):
        p = tmp_path / name
        p.write_bytes(data)
        files.append(p)
        return p

    goods = {"le": _hdat(), "be": _hdat(big=True), "split": _hdat(split=24), "lamax0": _hdat(lamax=0)}
    for name, data in goods.items():
        valid.append(put(f"good_{name}", data))
    rng = np.random.default_rng(1909)
    base = goods["le"]
    for cut in range(0, len(base), 7):                          # every truncation, 7-byte steps
        put(f"cut_{cut}", base[:cut])
    for k in range(300):                                       # seeded byte flips
        b = bytearray(base)
        for _ in range(1 + k % 3):
            b[int(rng.integers(0, len(b)))] = int(rng.integers(0, 256))
        put(f"flip_{k}", bytes(b))
    for off in range(0, min(len(base), 400), 4):               # extreme 4-byte fields over the first records
        for v in (-1, 0, 1 << 30, 2 ** 31 - 1, -(2 ** 31)):
            b = bytearray(base)
            b[off:off + 4] = struct.pack("<i", v)
            put(f"int_{off}_{v & 0xffffffff}", bytes(b))
    put("empty", b"")
    put("marker_only", struct.pack("<i", 8))
    out = {ln.split(" ", 1)[0]: ln for ln in _run(harness, "hdat", files)}
    assert len(out) == len(files)
    for p in valid:  # the valid files read through: two symmetries, then the end
        ln = out[str(p)]
        assert ln.startswith(f"{p} open 0") and " sym 2 arrays 0 desc 0" in ln and ln.endswith("next -4"), ln
    # a truncation inside a record is refused (at open or at the symmetry it
    # cuts); one at a record boundary leaves a shorter file that may be valid
    bounds, pos = {0}, 0
    while pos < len(base):
        pos += 8 + struct.unpack_from("<i", base, pos)[0]
        bounds.add(pos)
    inside = [cut for cut in range(0, len(base), 7) if cut not in bounds]
    assert len(inside) > 100
    for cut in inside:
        ln = out[str(tmp_path / f"cut_{cut}")]
        assert " open -6" in ln or ln.endswith("next -6"), ln


def test_sizeh_reader_under_sanitizers(harness, tmp_path):
    good = ("NCHAN =   12  NCON =     240 MNP2 =    250  S=  2  L=  3 PI=  1\n"
            "NCHAN =    7  NCON =     140 MNP2 =    151  S=  4  L=  0 PI=  0\n")
    texts = {"good": good, "empty": "", "short": "NCHAN =  1\n", "letters": good.replace("240", "2x0"),
             "long": "9" * 100000 + "\n", "nonl": good.rstrip("\n"), "many": good * 40,
             "neg": good.replace("  12", " -12"), "nul": good[:20] + "\0" + good[21:]}
    files = []
    for name, t in texts.items():
        p = tmp_path / f"sizeh_{name}"
        p.write_text(t)
        files.append(p)
    lines = _run(harness, "sizeh", files + [tmp_path / "missing"])
    assert len(lines) == 2 * (len(files) + 1)
    got = {(ln.split()[0].rsplit("/", 1)[-1], int(ln.split()[3])): (int(ln.split()[5]), int(ln.split()[7]))
           for ln in lines}
    assert got[("sizeh_good", 0)] == (0, 2) and got[("sizeh_nonl", 0)] == (0, 2)
    assert got[("sizeh_many", 0)] == (0, 80)  # 80 rows counted, 4 stored
    assert got[("sizeh_empty", 0)] == (0, 0)
    assert got[("sizeh_letters", 0)] == (-6, 0) and got[("sizeh_long", 0)] == (-6, 0)
    assert got[("sizeh_good", 1)][0] == -6  # sizeH columns read as sizeBP: not integers
    assert got[("missing", 0)][0] == -6


def test_omega_writer_under_sanitizers(harness, tmp_path):
    lines = _run(harness, "omega", [tmp_path])
    assert len(lines) == 3 * 2 * 5 * 2 * 2
    assert all(ln.endswith("status 0") for ln in lines), [ln for ln in lines if not ln.endswith("status 0")]
