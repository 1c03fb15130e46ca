"""Host C code under AddressSanitizer and UndefinedBehaviorSanitizer: the
oracle and the CPU row-form comparator are rebuilt with both sanitizers
(halting on the first report) into a small driver (tests/san_driver.c) and
run on the degenerate-input batch and on synthetic batches; their results
must equal those of the regular builds."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import cpu_rowform
import oracle
import synth
from edge_batch import edge_pairs, make_batch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
SOURCES = {
    "oracle": (os.path.join(ROOT, "oracle", "phmm_oracle.c"), ["-O1", "-ffp-contract=off",
                                                                 "-DUSE_ORACLE"]),
    "rowform": (os.path.join(ROOT, "cpu_rowform", "rowform.c"), ["-O1", "-mavx2", "-mfma",
                                                                  "-fopenmp", "-DUSE_ROWFORM"]),
}
KEYS = ("reads", "base_quals", "ins_quals", "del_quals", "gcp", "read_offsets", "haplotypes",
        "hap_offsets", "pair_list")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    out = {}
    for name, (src, flags) in SOURCES.items():
        exe = str(d / ("san_" + name))
        subprocess.run(["gcc", "-std=gnu11", *SAN, *flags, os.path.join(HERE, "san_driver.c"),
                        src, "-o", exe, "-lm"], check=True)
        out[name] = exe
    return out


def run_driver(exe, batch, d):
    os.makedirs(d, exist_ok=True)
    for k in KEYS:
        np.ascontiguousarray(batch[k]).tofile(os.path.join(d, k + ".bin"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe, d], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    return np.fromfile(os.path.join(d, "out.bin"), np.float64)


def batches():
    yield "edge", make_batch(edge_pairs())
    yield "batched_uneven", synth.generate("batched_uneven", 4, 2)
    yield "long_reads", synth.generate("long_reads", 0, 1)


@pytest.mark.parametrize("name", ["edge", "batched_uneven", "long_reads"])
def test_sanitized_oracle_and_rowform(drivers, tmp_path, name):
    b = dict(batches())[name]
    if name == "long_reads":  # one 10 kbp pair keeps the sanitized run short
        b["pair_list"] = np.ascontiguousarray(b["pair_list"][:1])
    got = run_driver(drivers["oracle"], b, str(tmp_path / "o"))
    want = oracle.forward_pairs(b, rescale=True)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    got = run_driver(drivers["rowform"], b, str(tmp_path / "r"))
    want, _ = cpu_rowform.forward_pairs(b, threads=2)
    fin = np.isfinite(want)
    assert np.array_equal(fin, np.isfinite(got))
    # FP32 rows: the sanitized build's code differs (-O1, instrumentation), so
    # the rounding of the FP32 results may differ by a few units in the last
    # place; accepted results stay within the FP32 bound of the oracle
    assert np.abs(got[fin] - want[fin]).max(initial=0) <= 1e-5
    ref = oracle.forward_pairs(b, rescale=True)
    assert np.abs(got[fin] - ref[fin]).max(initial=0) <= 1e-4


# ---------------------------------------------------------------- host runtime
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CSRC = os.path.join(ROOT, "paper_2606_25738_amd", "csrc")
LIB_SOURCES = ["phmm_api.hip", "phmm_pack.hip", "phmm_short.hip", "phmm_long.hip", "phmm_peak.hip",
               "phmm_server.hip", "phmm_genotype.hip"]
# the sanitizers instrument the host pass only (-Xarch_host before each)
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]


@pytest.fixture(scope="module")
def host_driver(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    d = tmp_path_factory.mktemp("sanhost")
    flags = ["--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", *HOST_SAN, "-Xclang",
             "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC]
    jobs = []
    objs = []
    for src in LIB_SOURCES + [os.path.join(HERE, "san_host_driver.cpp")]:
        obj = str(d / (os.path.basename(src) + ".o"))
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        jobs.append(subprocess.Popen([HIPCC, *flags, "-c", path, "-o", obj],
                                     stdout=subprocess.PIPE, stderr=subprocess.PIPE))
        objs.append(obj)
    for j in jobs:
        _, err = j.communicate()
        assert j.returncode == 0, err.decode()[-3000:]
    exe = str(d / "san_host_driver")
    subprocess.run([HIPCC, "--offload-arch=gfx950", *HOST_SAN, *objs, "-o", exe], check=True,
                   capture_output=True)
    return exe


def host_run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    return r.stdout


def mutations():
    b = make_batch(edge_pairs())
    yield "valid", b
    m = dict(b, reads=b["reads"].copy())
    m["reads"][37] = ord("x")
    yield "bad read base", m
    m = dict(b, haplotypes=b["haplotypes"].copy())
    m["haplotypes"][len(m["haplotypes"]) - 1] = ord("U")
    yield "bad hap base (last byte)", m
    m = dict(b, read_offsets=b["read_offsets"].copy())
    m["read_offsets"][3] = m["read_offsets"][2]
    yield "empty read", m
    m = dict(b, hap_offsets=b["hap_offsets"].copy())
    m["hap_offsets"][5] = m["hap_offsets"][6] + 1
    yield "offsets not increasing", m
    m = dict(b, pair_list=b["pair_list"].copy())
    m["pair_list"][4, 0] = 13
    yield "read index out of range", m
    m = dict(b, pair_list=b["pair_list"].copy())
    m["pair_list"][12, 1] = 1 << 31
    yield "hap index out of range", m
    big = make_batch([(b"A" * 131073, b"ACGT", 30, 45, 45, 10)])
    yield "read too long", big


def test_sanitized_host_validation(host_driver, tmp_path):
    """phmm_validate_batch of an instrumented build on valid and malformed
    batches: no sanitizer report, and the same code, lengths and message as
    the regular library."""
    import paper_2606_25738_amd as phmm
    for i, (what, b) in enumerate(mutations()):
        d = str(tmp_path / ("m%d" % i))
        os.makedirs(d)
        for k in KEYS:
            np.ascontiguousarray(b[k]).tofile(os.path.join(d, k + ".bin"))
        rc, ml, mk, msg = host_run(host_driver, "validate", d).rstrip("\n").split(" ", 3)
        try:
            want = (0,) + phmm.phmm_validate_batch(b)
            want_msg = None
        except phmm.PhmmError as e:
            want = (e.code,)
            want_msg = str(e)
        assert int(rc) == want[0], what
        if want[0] == 0:
            assert (int(ml), int(mk)) == want[1:], what
        else:
            assert msg in want_msg, (what, msg, want_msg)


def test_sanitized_host_options(host_driver):
    """Option checks run before any device work: every bad option is
    PHMM_EINVAL naming the option (the accept_min_sum floor of 1e-30
    included), with no sanitizer report and no context returned."""
    out = host_run(host_driver, "options").strip().splitlines()
    assert len(out) == 9
    for line in out:
        what, rc, msg, null = line.split("|")
        assert int(rc) == -1 and null == "1", line
        assert what.split()[0] in msg, line
