"""Host check of every index range the HIP kernels form from the plan.

tests/plan_check.cpp is compiled with g++ against the library's planner
(paper_1409_0297_amd/csrc/plan.cpp) and run for the geometries the GPU tests
and the benchmark use, single problems and batches.  It checks the front
arena, solve-vector, permutation, diagonal-block-inverse, inverse-work and
gather ranges (inside their buffers, pairwise disjoint where each has one
owner), the boundary-to-parent maps and the assembly blocks.  A diagonal-
block slot past the end of its buffer is the access that once faulted the
GPU during the batched setup; it is one of the checks.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1409_0297_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("plan") / "plan_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I" + CSRC, os.path.join(ROOT, "tests", "plan_check.cpp"),
                    os.path.join(CSRC, "plan.cpp"), "-o", exe], check=True)
    return exe


def run(exe, *geoms, streamed=False, points=False, nc=1):
    r = subprocess.run([exe] + (["-s"] if streamed else []) + (["-p"] if points else [])
                       + (["-c", str(nc)] if nc > 1 else [])
                       + [",".join(map(str, g)) for g in geoms], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr
    return r.stdout


OCT, BIS = 0, 1


@pytest.mark.parametrize("geom", [
    (2, 32, 8, OCT), (2, 64, 8, OCT), (2, 64, 8, BIS), (2, 48, 6, OCT), (2, 128, 8, OCT),
    (2, 512, 16, OCT), (2, 256, 16, OCT), (2, 192, 12, OCT),
    (3, 12, 3, OCT), (3, 12, 3, BIS), (3, 24, 6, BIS), (3, 48, 6, OCT)])
def test_single_problem_plans(checker, geom):
    out = run(checker, geom)
    if geom[0] == 2 and geom[1] <= 64:
        assert "P entries checked" in out


def test_uneven_2d_batch(checker):
    run(checker, (2, 48, 6, OCT), (2, 32, 8, OCT), (2, 32, 8, OCT), (2, 64, 8, OCT))


def test_schrodinger_family_batch(checker):
    # the 48-problem family: 16 each of 128^2 / b 8, 192^2 / b 12, 256^2 / b 16
    geoms = [((2, 128, 8, OCT), (2, 192, 12, OCT), (2, 256, 16, OCT))[i % 3] for i in range(48)]
    out = run(checker, *geoms)
    assert "fronts" in out


def test_3d_batch(checker):
    run(checker, (3, 12, 3, OCT), (3, 8, 4, OCT))


@pytest.mark.parametrize("geom", [(3, 12, 3, BIS), (3, 16, 4, BIS), (3, 24, 6, BIS), (3, 32, 4, BIS), (3, 48, 6, OCT),
                                  (2, 64, 8, OCT), (2, 512, 16, OCT)])
def test_streamed_storage_plans(checker, geom):
    """Streamed storage: two adjacent levels never share arena space and the
    compact factors do not overlap."""
    run(checker, geom, streamed=True)


def test_streamed_batch(checker):
    run(checker, (2, 48, 6, OCT), (2, 32, 8, OCT), (2, 64, 8, OCT), streamed=True)


def test_3d_128_bisection_plan(checker):
    """The 3D Helmholtz configuration's plan (128^3, b = 8, bisection,
    streamed): 8191 fronts up to 48896, every kernel range checked."""
    out = run(checker, (3, 128, 8, BIS), streamed=True)
    assert "fronts 8191" in out and "max_front 48896" in out, out


@pytest.mark.parametrize("geom", [(2, 32, 8, OCT), (2, 64, 8, OCT), (3, 12, 3, BIS), (2, 512, 16, OCT)])
def test_point_pattern_plans(checker, geom):
    """Point stencil pattern (every point its own set): same fronts, one
    assembly block per point, every entry of P assembled once."""
    out = run(checker, geom, points=True)
    if geom[1] <= 64:
        assert "P entries checked" in out


def test_bad_geometry_is_reported(checker):
    r = subprocess.run([checker, "2,30,8,0"], capture_output=True, text=True)
    assert r.returncode == 1 and "FAIL" in r.stdout


@pytest.mark.parametrize("geom", [(2, 16, 4, OCT), (2, 64, 16, OCT), (2, 64, 8, OCT), (2, 128, 16, OCT),
                                  (3, 8, 4, OCT), (3, 12, 3, BIS), (3, 20, 5, OCT)])
def test_vector_field_plans(checker, geom):
    """Maxwell plans: d unknowns per point (expand_plan)."""
    out = run(checker, geom, nc=geom[0])
    if geom[0] == 2 and geom[1] <= 64:
        assert "P entries checked" in out
