"""Host-side bounds check of the scoring kernels' LDS row staging (CPU only).

tests/staging_check.cpp replays every copy of every staging step through the
library's own geometry functions (staging_geom.h: make_staging, for_each_copy,
zero_slot_rel) and checks every global read, every LDS write, the zero-slot
owners and what each gather can reach.  The planted variants show the check
is sharp: each reintroduces a plausible mistake in a copy of the header and
must be reported.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_20891_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "staging_check.cpp")


def _build_and_run(tmp_path, header_text=None):
    inc = str(tmp_path / "inc")
    os.makedirs(inc, exist_ok=True)
    hdr = open(os.path.join(CSRC, "staging_geom.h")).read() if header_text is None else header_text
    with open(os.path.join(inc, "staging_geom.h"), "w") as f:
        f.write(hdr)
    exe = str(tmp_path / "staging_check")
    subprocess.run(["g++", "-std=c++17", "-O2", "-I", inc, SRC, "-o", exe], check=True,
                   capture_output=True, text=True)
    return subprocess.run([exe], capture_output=True, text=True, timeout=300)


@pytest.fixture(scope="module")
def header():
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    return open(os.path.join(CSRC, "staging_geom.h")).read()


def test_staging_geometry_in_bounds(tmp_path, header):
    res = _build_and_run(tmp_path, header)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-2000:]
    assert res.stdout.startswith("ok "), res.stdout


PLANTED = {
    # four waves copying with the eight-wave chunk stride: chunks are skipped
    "four_waves_eight_wave_stride": [("SCORE_THREADS = 512", "SCORE_THREADS = 256"),
                                     ("c += SCORE_WAVES", "c += 8")],
    # the final chunk without its clamp: lanes read past the block
    "no_last_chunk_clamp": [("return lane_off < lim ? lane_off : lim;", "return lane_off;")],
    # the final chunk given to the wrong wave: its slot owner no longer matches
    "last_chunk_wrong_owner": [("if (chunk_owner(last) == wave)", "if (chunk_owner(last + 1) == wave)")],
    # zero slots never re-zeroed after a copy overwrote them
    "no_slot_owner": [("(uint64_t)chunk_owner(rel >> STAGE_CHUNK_LOG2) : 0xffull", "0xffull : 0xffull")],
    # halves one chunk too short
    "half_too_short": [("stage_round_up((size_t)G * pitch_bytes, STAGE_CHUNK)",
                        "stage_round_up((size_t)G * pitch_bytes, STAGE_CHUNK) - STAGE_CHUNK")],
}


@pytest.mark.parametrize("name", sorted(PLANTED))
def test_planted_staging_mistake_is_reported(tmp_path, header, name):
    text = header
    for old, new in PLANTED[name]:
        assert old in text, (name, old)
        text = text.replace(old, new)
    res = _build_and_run(tmp_path, text)
    assert res.returncode != 0 and "FAIL" in res.stdout + res.stderr, (name, res.stdout[-500:])
