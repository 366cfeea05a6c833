"""The C example client (paper_1501_03879_amd/examples/nlem_client.c, built
with the library): NLEM through the C ABI from a C program, a child process
with no Python or torch in it, checked against the FP64 oracle at a fixed
iteration count (1e-4 of the intensity range, every pixel, and every pixel's
iteration count)."""

import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from helpers import rel_errors, report

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLIENT = os.path.join(ROOT, "paper_1501_03879_amd", "examples", "nlem_client")


def test_c_client_matches_oracle(tmp_path):
    assert os.path.exists(CLIENT), "the C client is built with the library (build())"
    H, W, pr, wr, T = 37, 45, 3, 10, 9
    rng = np.random.default_rng(81)
    img = synth.add_gaussian_noise(rng, synth.piecewise_smooth_image(rng, H, W), 20.0).astype(np.float32)
    inp, outp, stp = tmp_path / "in.f32", tmp_path / "out.f32", tmp_path / "stats.bin"
    img.tofile(inp)
    args = [CLIENT, str(inp), str(H), str(W), str(pr), str(wr), "200", "0", "255", "0.001", str(T), "0",
            str(outp), str(stp)]
    print("[c-client]", " ".join(args[1:]), flush=True)
    r = subprocess.run(args, capture_output=True, text=True, timeout=120)
    print(r.stdout.strip(), r.stderr.strip(), flush=True)
    assert r.returncode == 0, r.stderr
    got = np.fromfile(outp, dtype=np.float32).astype(np.float64)
    st = np.fromfile(stp, dtype=np.int32).reshape(-1, 4)
    ref = oracle.nlem(img, pr, wr, 200.0, 0.0, 255.0, 1e-3, T, 0.0)
    e, rr = rel_errors(got, ref["out"], 255.0)
    report(f"C client nlem r{pr} R{wr} T{T}", e, rr)
    assert got.shape == (H * W,) and e <= 1e-4
    assert np.all(st[:, 0] == T)


def test_c_client_reports_bad_arguments(tmp_path):
    """A library argument error reaches the C caller as a status (exit 4)."""
    assert os.path.exists(CLIENT)
    img = np.zeros((8, 8), np.float32)
    inp = tmp_path / "in.f32"
    img.tofile(inp)
    # rho = 0 is rejected before any launch
    r = subprocess.run([CLIENT, str(inp), "8", "8", "1", "2", "10", "0", "255", "0", "5", "0",
                        str(tmp_path / "o.f32")], capture_output=True, text=True, timeout=120)
    assert r.returncode == 4 and "EM_ERR_INVALID_ARG" in r.stderr, (r.returncode, r.stderr)
