"""Host build of the device construction of the sweep (csrc/wg_construct.h:
float64 with an error bound, double words with an error bound, exact
integers) against the library's exact host construction (big integers, which
test_abi_host pins to the rational oracle), entry for entry, on point sets of
every kind (Sections 4.1, 4.2).  Needs hipcc (no GPU)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-std=c++17", "-O2", "-ffp-contract=off", "-I", os.path.join(ROOT, "paper_2201_10369_amd", "csrc"),
         "-I", os.path.join(ROOT, "include")]


@pytest.fixture(scope="module")
def check_binary(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("construct_check")
    objs = []
    for src, lang in (("tests/native/construct_check.cpp", ["-x", "hip", "--offload-arch=gfx950"]),
                      ("paper_2201_10369_amd/csrc/exact_construct.cpp", ["-x", "c++"])):
        obj = str(out / (os.path.basename(src) + ".o"))
        subprocess.run([HIPCC, *FLAGS, *lang, "-c", os.path.join(ROOT, src), "-o", obj], check=True,
                       capture_output=True, text=True)
        objs.append(obj)
    exe = str(out / "construct_check")
    subprocess.run([HIPCC, "--offload-arch=gfx950", *objs, "-o", exe], check=True, capture_output=True, text=True)
    return exe


def test_device_construction_host_build_matches_exact(check_binary):
    res = subprocess.run([check_binary, "150"], check=True, capture_output=True, text=True, timeout=600)
    rows = [l for l in res.stdout.splitlines() if l.startswith("F(")]
    assert len(rows) == 12 * 8
    pat = re.compile(r"F\((\d),(\d)\) (\w+) sets (\d+) f64 (\d+) dw (\d+) singular (\d+) mismatch (\d+) "
                     r"status (\d+) toobig (\d+)")
    f64_short = 0
    for line in rows:
        m, r, cat, sets, f64, dw, sing, mism, status, toobig = pat.match(line).groups()
        assert int(mism) == 0 and int(status) == 0, line          # no tier ever decides wrongly
        assert int(toobig) == 0, line
        valid = int(sets) - int(sing)
        assert int(dw) == valid, line                             # double words decide all these
        if cat in ("family", "random", "pairs", "dyadic", "cancel", "quarter"):
            # float64 with a bound decides nearly all of these (it leaves an
            # entry only when the value lies near a float32 rounding boundary)
            assert int(f64) >= 0.95 * valid, line
        f64_short += valid - int(f64)
    assert f64_short > 0                                          # the double-word tier was exercised
