"""Mutation testing of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of the oracle (a dropped term, a
wrong sign, swapped operands, a transposed matrix, a wrong constant or boundary) and
runs the pin tests that cover that part of the oracle against the copy: every
mutant must fail at least one of them.  A mutant that survives names a mistake the
pins cannot see.  The copies live in a temporary directory; the cases run in
parallel, a few seconds each.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow

CPP = "oracle/gs2d_oracle.cpp"
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_scale.py"]
DEPTH = ["tests/test_oracle_depth_variants.py"]
MAPLOSS = ["tests/test_oracle_mapping_loss.py"]
LOSS = ["tests/test_oracle_se3_loss.py", "tests/test_oracle_depth_variants.py"]

# (name, file, original text, mutated text, pin tests that must catch it)
MUTANTS = [
    # the rasterizer: forward, backward, pose gradient
    ("normal chain of t_u dropped", CPP,
     "for (int cc = 0; cc < 3; ++cc) gtuc[cc] = s.su * ga[cc] + tmp[cc];",
     "for (int cc = 0; cc < 3; ++cc) gtuc[cc] = s.su * ga[cc];", PINS),
    ("sign of d(u, v)/d q2", CPP,
     "-(gu * h.q[0] + gv * h.q[1]) / (h.q[2] * h.q[2])", "(gu * h.q[0] + gv * h.q[1]) / (h.q[2] * h.q[2])", PINS),
    ("cross-product operands swapped", CPP, "cross(h.hv, gq, ghu);", "cross(gq, h.hv, ghu);", PINS),
    ("stop rule on the incoming transmittance", CPP, "if (Tn < sc.k.t_min) break;", "if (T < sc.k.t_min) break;",
     PINS),
    ("order by index instead of depth", CPP, "return sc.surf[(size_t)a].key < sc.surf[(size_t)b].key;",
     "return a < b;", PINS),
    ("K^T without its principal-point terms", CPP, "gA[2][j] = cam.cx * m0 + cam.cy * m1 + m2;",
     "gA[2][j] = m2;", PINS),
    ("R instead of R^T to the world frame", CPP,
     "gmu_w[cc] = R[0 * 4 + cc] * gmu[0] + R[1 * 4 + cc] * gmu[1] + R[2 * 4 + cc] * gmu[2];",
     "gmu_w[cc] = R[cc * 4 + 0] * gmu[0] + R[cc * 4 + 1] * gmu[1] + R[cc * 4 + 2] * gmu[2];", PINS),
    ("clamped opacity passes its derivative", CPP, "if (!h.clamped) {", "if (true) {", PINS),
    ("Gaussian exp(-rho) instead of exp(-rho/2)", CPP, "h.G = std::exp(-0.5 * h.rho);", "h.G = std::exp(-h.rho);",
     PINS),
    ("filter scale dropped in the backward", CPP, "double gcx = -2.0 * kk.filter_scale * h.dx * dL_drho;",
     "double gcx = -2.0 * h.dx * dL_drho;", PINS),
    ("alpha derivative without 1/(1 - alpha)", CPP,
     "suffix[(size_t)(8 * (i + 1) + ch)] / (1.0 - h.alpha));", "suffix[(size_t)(8 * (i + 1) + ch)]);", PINS),
    ("normal t_v x t_u", CPP, "cross(s.tuc, s.tvc, s.n);", "cross(s.tvc, s.tuc, s.n);", PINS),
    ("pose rotation without the normal term", CPP, "pose[3 + cc] = c1[cc] + c2[cc] + c3[cc] + c4[cc];",
     "pose[3 + cc] = c1[cc] + c2[cc] + c3[cc];", PINS),
    ("pose sign mu_c x g swapped", CPP, "cross(s.mu_c, gmu, c1);", "cross(gmu, s.mu_c, c1);", PINS),
    ("weight with the outgoing transmittance", CPP, "    double w = h.alpha * T;\n",
     "    double w = h.alpha * Tn;\n", PINS),
    ("s_u gradient against t_v", CPP, "double gsu = dot(s.tuc, ga), gsv = dot(s.tvc, gb);",
     "double gsu = dot(s.tvc, ga), gsv = dot(s.tvc, gb);", PINS),
    ("f_x for f_y in the homography", CPP, "s.M[1][j] = cam.fy * col[j][1] + cam.cy * col[j][2];",
     "s.M[1][j] = cam.fx * col[j][1] + cam.cy * col[j][2];", PINS),
    ("filter branch with the intersection's depth", CPP, "    h.rho = rho2d;\n    h.d = s.M[2][2];",
     "    h.rho = rho2d;\n    h.d = s.M[2][0] * h.u + s.M[2][1] * h.v + s.M[2][2];", PINS),
    # depth variants
    ("median on T >= 1/2", CPP, "if (e.T > 0.5) med = e.h.d;", "if (e.T >= 0.5) med = e.h.d;", DEPTH),
    ("median at the first crossing", CPP, "if (e.T > 0.5) med = e.h.d;",
     "if (e.T > 0.5 && med == 0.0) med = e.h.d;", DEPTH),
    ("median on the outgoing transmittance", CPP, "if (e.T > 0.5) med = e.h.d;",
     "if (e.T * (1.0 - e.h.alpha) > 0.5) med = e.h.d;", DEPTH),
    ("D instead of D / O", CPP, "depth_norm[p] = out[7] > 0.0 ? out[3] / out[7] : 0.0;",
     "depth_norm[p] = out[3];", DEPTH),
    ("margin ignores the median", CPP, "fm = std::min(fm, rel(e.T, 0.5));", "(void)0;", DEPTH),
    # the mapping loss
    ("SSIM C1", "oracle/mapping_loss.py", "C1 = 0.01 ** 2", "C1 = 0.02 ** 2", MAPLOSS),
    ("SSIM C2", "oracle/mapping_loss.py", "C2 = 0.03 ** 2", "C2 = 0.01 ** 2", MAPLOSS),
    ("SSIM sigma", "oracle/mapping_loss.py", "SIGMA = 1.5", "SIGMA = 2.0", MAPLOSS),
    ("SSIM window size", "oracle/mapping_loss.py", "WINDOW = 11", "WINDOW = 9", MAPLOSS),
    ("depth-normal cross product order", "oracle/mapping_loss.py", "c = torch.linalg.cross(dx, dy, dim=0)",
     "c = torch.linalg.cross(dy, dx, dim=0)", MAPLOSS),
    ("forward difference", "oracle/mapping_loss.py", "dx = X[:, 1:-1, 2:] - X[:, 1:-1, :-2]",
     "dx = X[:, 1:-1, 2:] - X[:, 1:-1, 1:-1]", MAPLOSS),
    ("f_x for f_y in the lifted points", "oracle/mapping_loss.py", "depth * (ys - cy) / fy", "depth * (ys - cy) / fx",
     MAPLOSS),
    ("variance without -mu^2", "oracle/mapping_loss.py", "vx = _local_mean(x * x, w) - mx * mx",
     "vx = _local_mean(x * x, w)", MAPLOSS),
    ("covariance mu_x mu_x", "oracle/mapping_loss.py", "cxy = _local_mean(x * y, w) - mx * my",
     "cxy = _local_mean(x * y, w) - mx * mx", MAPLOSS),
    ("sign of L_n", "oracle/mapping_loss.py", "ln = 1.0 - (depth_normals(D, camera) * N).sum(dim=0)",
     "ln = 1.0 + (depth_normals(D, camera) * N).sum(dim=0)", MAPLOSS),
    ("SSIM summed over channels", "oracle/mapping_loss.py", "dssim = 1.0 - ssim_map(I, It).mean(dim=0)",
     "dssim = 1.0 - ssim_map(I, It).sum(dim=0)", MAPLOSS),
    ("L1 averaged over channels", "oracle/mapping_loss.py", "l1 = (I - It).abs().sum(dim=0)",
     "l1 = (I - It).abs().mean(dim=0)", MAPLOSS),
    ("shifted border", "oracle/mapping_loss.py", "torch.nn.functional.pad(inner, (1, 1, 1, 1))",
     "torch.nn.functional.pad(inner, (2, 0, 1, 1))", MAPLOSS),
    ("unnormalised window", "oracle/mapping_loss.py", "g = g / g.sum()", "g = g", MAPLOSS),
    ("normal term dropped", "oracle/mapping_loss.py", "per_pixel = w_l1 * l1 + w_ssim * dssim + w_d * ld + w_n * ln",
     "per_pixel = w_l1 * l1 + w_ssim * dssim + w_d * ld", MAPLOSS),
    # the tracking loss's masks
    ("opacity mask threshold", "oracle/loss.py", "OPACITY_MASK = 0.95", "OPACITY_MASK = 0.9", LOSS),
    ("normal mask sign", "oracle/loss.py", "m_n = ndotr > 0", "m_n = ndotr < 0", LOSS),
]


def _copy_tree(dst: str):
    ignore = shutil.ignore_patterns("*.so", "*.so.tmp*", "__pycache__")
    for d in ("oracle", "synth"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(dst, d), ignore=ignore)
    os.makedirs(os.path.join(dst, "tests"))
    for f in os.listdir(os.path.join(ROOT, "tests")):
        src = os.path.join(ROOT, "tests", f)
        if f == "golden":
            shutil.copytree(src, os.path.join(dst, "tests", f))
        elif f.endswith(".py"):
            shutil.copy(src, os.path.join(dst, "tests", f))


def _run_mutant(case) -> tuple:
    name, path, old, new, tests = case
    with tempfile.TemporaryDirectory(prefix="gs2d_mutant_") as tmp:
        _copy_tree(tmp)
        target = os.path.join(tmp, path)
        with open(target) as f:
            text = f.read()
        if text.count(old) != 1:
            return name, "site", f"the original text occurs {text.count(old)} times"
        with open(target, "w") as f:
            f.write(text.replace(old, new))
        env = {k: v for k, v in os.environ.items() if k not in ("PYTHONPATH", "GS2D_ORACLE_SANITIZED")}
        env["OMP_NUM_THREADS"] = "2"
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *tests], cwd=tmp,
                           env=env, capture_output=True, text=True, timeout=600)
        out = r.stdout + r.stderr
        tail = out.strip().splitlines()[-1] if out.strip() else ""
        if r.returncode == 1 and "failed" in tail:
            return name, "killed", tail
        return name, "survived" if r.returncode == 0 else "error", out[-2000:]


def test_every_mutant_fails_a_pin(oracle_mod):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    workers = max(1, min(8, (os.cpu_count() or 2) // 2))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(_run_mutant, MUTANTS))
    for name, verdict, detail in results:
        print(f"{verdict:8s} {name}: {detail.splitlines()[-1] if detail else ''}")
    bad = [(n, v, d) for n, v, d in results if v != "killed"]
    assert not bad, "\n\n".join(f"{n} [{v}]\n{d}" for n, v, d in bad)
