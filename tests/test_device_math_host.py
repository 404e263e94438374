"""Host build of the library's per-element math (no GPU): the closed-form PSD projection of the
Neo-Hookean dP/dF (singular value decomposition of F, twist/flip modes and a 3x3 scaling block)
against numpy's symmetric eigendecomposition of the same 9x9 matrix, clamped at zero."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2503_05020_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include "device_math.h"
#include <cstdio>
int main() {
  double F[9], mu, la;
  while (scanf("%lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf", &F[0], &F[1], &F[2], &F[3], &F[4], &F[5], &F[6],
               &F[7], &F[8], &mu, &la) == 11) {
    double Hs[45];
    ipcdev::nh_dPdF_projected(F, log(ipcdev::det33(F)), mu, la, Hs);
    for (int k = 0; k < 45; ++k) printf("%.17g%c", Hs[k], k == 44 ? '\n' : ' ');
  }
}
"""


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("device_math")
    src = d / "projection.cpp"
    src.write_text(PROGRAM)
    out = d / "projection"
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-I", CSRC, str(src), "-o", str(out)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return str(out)


def dPdF(F, mu, la):
    """mu d_ik d_jl + (mu - la ln J) G_il G_kj + la G_ij G_kl with G = F^-T, row-major (i,j),(k,l)."""
    G = np.linalg.inv(F).T
    c1 = mu - la * np.log(np.linalg.det(F))
    H = np.zeros((9, 9))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for m in range(3):
                    H[3 * i + j, 3 * k + m] = (mu if (i == k and j == m) else 0.0) + c1 * G[i, m] * G[k, j] \
                        + la * G[i, j] * G[k, m]
    return H


def unpack(Hs):
    H = np.zeros((9, 9))
    t = 0
    for r in range(9):
        for c in range(r, 9):
            H[r, c] = H[c, r] = Hs[t]
            t += 1
    return H


def test_closed_form_projection_matches_eigh(exe):
    rng = np.random.default_rng(7)
    cases = []
    while len(cases) < 300:
        kind = len(cases) % 4
        if kind == 0:  # general deformation
            F = np.eye(3) * np.exp(rng.normal(0, 0.4)) + 0.4 * rng.normal(size=(3, 3))
        elif kind == 1:  # uniform compression or stretch
            F = np.eye(3) * np.exp(rng.normal(0, 0.6))
        elif kind == 2:  # two nearly equal singular values
            U, _ = np.linalg.qr(rng.normal(size=(3, 3)))
            V, _ = np.linalg.qr(rng.normal(size=(3, 3)))
            s = np.exp(rng.normal(0, 0.3, 3))
            s[1] = s[0] * (1 + 1e-9 * rng.normal())
            F = U @ np.diag(s) @ V.T
        else:  # strongly anisotropic
            F = np.diag(np.exp(rng.normal(0, 1.0, 3))) @ np.linalg.qr(rng.normal(size=(3, 3)))[0]
        if np.linalg.det(F) <= 0:
            F[:, 0] *= -1
        mu = 1e5 * np.exp(rng.normal())
        la = mu * (1 + 4 * abs(rng.normal()))
        cases.append((F, mu, la))
    text = "\n".join(" ".join(f"{v:.17g}" for v in list(F.ravel()) + [mu, la]) for F, mu, la in cases)
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout.split("\n")
    worst, clamped = 0.0, 0
    for (F, mu, la), line in zip(cases, out):
        H = dPdF(F, mu, la)
        w, V = np.linalg.eigh(H)
        clamped += int(w.min() < 0)
        expected = (V * np.maximum(w, 0.0)) @ V.T
        got = unpack(np.array([float(v) for v in line.split()]))
        worst = max(worst, np.abs(got - expected).max() / np.linalg.norm(H))
    assert clamped > 50, "the cases must exercise the clamping"
    assert worst <= 1e-10, worst
