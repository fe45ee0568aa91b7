"""Host-side behaviour that needs no GPU: the benchmark's one-GPU contract and
the seeded workload generators."""
import os
import subprocess
import sys

import numpy as np

from paper_1703_07206_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_workloads_are_seeded_and_shaped():
    a, b = W.poisson2d_sine(n=5), W.poisson2d_sine(n=5)
    assert np.array_equal(a.f, b.f) and a.f.shape == (33, 33)
    assert W.poisson2d_sine(n=5, seed=9).f.tolist() != a.f.tolist()
    blobs = W.poisson2d_blobs(n=6)
    assert blobs.faces == "DDNN" and blobs.f.shape == (65, 65)
    sph = W.helmholtz3d_spheres(n=4)
    assert sph.sigma.min() == 1.0 and 2.0 <= sph.sigma.max() <= 80.0
    assert np.all(sph.G[0] == -1.0) and np.all(sph.G[-1] == 1.0) and sph.a == -0.5
    adj = W.helmholtz3d_adjoint(n=4)
    assert np.array_equal(adj.sigma, W.sphere_medium(4, 3))  # same medium as the forward problem
    assert adj.extra["fd_f"].shape == (10, 3) and adj.extra["fd_eps"].min() >= 1
    ch = W.poisson3d_charges(n=4)
    assert ch.f.shape == (17, 17, 17) and "u_target" in ch.extra
    cap = W.capacitor_tanh(n=4, sign=-1)
    assert cap.faces == "NNNNDD" and 0.1 <= cap.sigma.min() and cap.sigma.max() <= 1.0


def test_poisson_workloads_use_the_papers_sign():
    # -lap(u) = f is handed over as lap(u) = -f: the sine source is negative inside
    wl = W.poisson2d_sine(n=5, noise=0.0)
    assert wl.f[16, 16] < 0 and abs(wl.f[16, 16] + 2 * np.pi ** 2) < 1e-12
