"""The benchmark's command-line contract that needs no GPU: more than one
GPU is refused with a message (there is no multi-GPU path), and the
algorithmic byte counts of the kernel classes are the documented ones."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_per_cell():
    sys.path.insert(0, ROOT)
    import bench
    T = 4
    b = bench.algorithmic_bytes_per_cell
    # FP32 multigrid values, one 8-byte operator record per cell
    assert b("rbgs_fine", T) == 20                 # x, b, operator in; x out
    assert b("rbgs_fine_dots", T) == 36            # + r, q (FP64)
    assert b("rbgs_fine_colour", T) == 14          # half of x, b, x out; every record
    assert b("mg_residual_fine", T) == 16.5        # x, b, operator in, coarse rhs out
    assert b("pcg_direction", T) == 76             # zT, p, x, diag, 3 faces in; p, q, x out
    assert b("pcg_update", T) == 28                # r, q in; r, b out
    assert b("local_solve", T) == 152 and b("local_solve", T, iso=True) == 96
    assert b("no_such_kernel", T) is None
    assert b("rbgs_fine", 8) == 56 and b("mg_residual_fine", 8) == 49  # FP64 levels
    assert b("rbgs_fine_colour", 8) == 40
    assert b("residual_schur", T) == 82 and b("residual_schur", 8) == 80


def test_step_bytes_formula():
    """Whole-step algorithmic bytes per cell: a linear iteration is the
    V(2,2) cycle (fine level 3 x 20 + 36 + 16.5 + 8.5 = 121 B in FP32; the
    coarser levels the same work on N/7 cells without dot products) plus the
    CG direction and update kernels; a step adds copies, the face limiter
    and one local solve + residual per evaluation."""
    sys.path.insert(0, ROOT)
    import bench
    lin32 = bench.linear_iteration_bytes(4)
    assert abs(lin32 - (121 + (4 * 20 + 16.5 + 8.5) / 7 + 76 + 28)) < 1e-12
    st = {"newton_its": 2, "ls_cuts": 1, "lin_its_total": 100}
    b = bench.step_bytes_per_cell(st, 4)
    evals = 4 * (152 + 82)
    assert abs(b - (96 + 62 + evals + 2 * 6 / 7 + 100 * lin32)) < 1e-9
    # FP64 V-cycles move about twice the FP32 bytes on the multigrid levels
    assert 1.6 < bench.linear_iteration_bytes(8) / lin32 < 2.0
