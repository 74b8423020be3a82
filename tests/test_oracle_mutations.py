"""Mutation check of the oracle's pins (CPU only).

Each entry below plants one plausible mistake in a copy of oracle/tt_oracle.c: a dropped term, a
flipped sign, a transposed operand, a wrong constant, a wrong tie rule, an off-by-one index. The
copy is compiled on its own and the pins in tests/test_oracle_pins.py run against it in a
subprocess (TT_ORACLE_LIB points the oracle's loader at the copy). Every copy must fail at least
one pin; an unmodified copy must pass them all, so that a broken harness cannot pass the check.
"""
import concurrent.futures
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "tt_oracle.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")

# (name, text in tt_oracle.c, replacement); each text occurs exactly once
MUTANTS = [
    # quaternion and dual-quaternion algebra (Sec. 2: warps as dual quaternions)
    ("qmul cross term sign", "double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];",
     "double x = a[0] * b[1] + a[1] * b[0] - a[2] * b[3] + a[3] * b[2];"),
    ("qrotate factor 2", "out[c] = p[c] + (2.0 / s) * (q[0] * up[c] + uup[c]);",
     "out[c] = p[c] + (1.0 / s) * (q[0] * up[c] + uup[c]);"),
    ("dq_apply dual scalar sign", "double X = w * up[c] + uup[c] + w * f[c] - e * u[c] + uf[c];",
     "double X = w * up[c] + uup[c] + w * f[c] + e * u[c] + uf[c];"),
    ("dq_apply drops u x f", "double X = w * up[c] + uup[c] + w * f[c] - e * u[c] + uf[c];\n    v[c]",
     "double X = w * up[c] + uup[c] + w * f[c] - e * u[c];\n    v[c]"),
    ("dq_apply_jac dX/de sign", "dXde[r] = -u[r];", "dXde[r] = u[r];"),
    ("dq_apply_jac transposed outer product", "- 2.0 * p[r] * u[c]", "- 2.0 * p[c] * u[r]"),
    ("dq_from_rt half", "dq[4 + c] = 0.5 * d[c];", "dq[4 + c] = d[c];"),
    ("dq_blend no sign alignment", "double sg = (d < 0.0) ? -1.0 : 1.0;", "double sg = 1.0;"),
    ("increment jacobian half", "Q[r * 6 + c] = 0.5 * Gr[r * 3 + c];", "Q[r * 6 + c] = Gr[r * 3 + c];"),
    ("increment jacobian lever sign", "Q[(4 + r) * 6 + c] = 0.5 * Gd[r * 3 + c] + 0.5 * gs;",
     "Q[(4 + r) * 6 + c] = 0.5 * Gd[r * 3 + c] - 0.5 * gs;"),
    ("quat_exp full angle", "q[0] = cos(0.5 * th);", "q[0] = cos(th);"),
    ("dq_normalize sign convention", "if (d[0] < 0.0)\n", "if (d[0] > 0.0)\n"),
    ("node-centred increment reversed", "t[c] = p[c] - Rp[c] + xi[3 + c];", "t[c] = Rp[c] - p[c] + xi[3 + c];"),
    # sampler and constants
    ("splitmix shift", "z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;", "z = (z ^ (z >> 26)) * 0x94D049BB133111EBULL;"),
    ("w_angle constant", "p->w_angle = 20.0;", "p->w_angle = 10.0;"),
    ("sampler seed offset", "uint64_t st = seed + GOLDEN64 * (uint64_t)(frame + 1);",
     "uint64_t st = seed + GOLDEN64 * (uint64_t)frame;"),
    ("fisher-yates range", "int j = i + (int)(r % (uint64_t)(Ku - i));", "int j = (int)(r % (uint64_t)Ku);"),
    # template: control points, blend weights, ARAP pair weights
    ("blend sigma", "alpha[t] = exp(-(bestd[t] - bestd[0]) / (2.0 * sbar * sbar));",
     "alpha[t] = exp(-(bestd[t] - bestd[0]) / (sbar * sbar));"),
    ("knn tie rule", "while (pos > 0 && (idx[pos - 1] < 0 || d < bestd[pos - 1])) pos--;",
     "while (pos > 0 && (idx[pos - 1] < 0 || d <= bestd[pos - 1])) pos--;"),
    ("arap weight sigma", "double sa = 2.0 * s->sbar;", "double sa = s->sbar;"),
    ("fps tie rule", "if (mind[j] > best) { best = mind[j]; bi = j; }", "if (mind[j] >= best) { best = mind[j]; bi = j; }"),
    ("sbar squared", "acc += sqrt(best);", "acc += best;"),
    ("arap weight sum over unordered pairs", "if (a != b) sa += arap_pair_weight(s, a, b);",
     "if (a < b) sa += arap_pair_weight(s, a, b);"),
    ("sparse graph and instead of or",
     "if (s->adj[(size_t)a * N + b] == 2 || s->adj[(size_t)b * N + a] == 2) {",
     "if (s->adj[(size_t)a * N + b] == 2 && s->adj[(size_t)b * N + a] == 2) {"),
    # frame: normals, matching, rotation fit, pre-selection (Sec. 2.1)
    ("backprojection fy", "P[1] = ((double)v - K->cy) / K->fy * z;", "P[1] = ((double)v - K->cy) / K->fx * z;"),
    ("normal orientation", "if (dot3(c, Pc) > 0.0)", "if (dot3(c, Pc) < 0.0)"),
    ("normal validity neighbour", "!depth_ok(depth[pix - W]) || ", ""),
    ("hamming tie rule", "if (d < best) { best = d; bi = b; }", "if (d <= best) { best = d; bi = b; }"),
    ("rotation fit no reflection fix", "double d = (det3(U) * det3(Vs) < 0.0) ? -1.0 : 1.0;", "double d = 1.0;"),
    ("rotation fit transposed", "Mx[3 * r + c] += w[k] * S2[3 * k + r] * S1[3 * k + c];",
     "Mx[3 * r + c] += w[k] * S1[3 * k + r] * S2[3 * k + c];"),
    ("eq4 weight squared", "w[k] = (d[k] > H) ? H / d[k] : 1.0;", "w[k] = (d[k] > H) ? (H / d[k]) * (H / d[k]) : 1.0;"),
    ("inlier count radius", "if (d[k] <= H) nin++;", "if (d[k] <= 2.0 * H) nin++;"),
    ("keep ratio", "if (hyp_W[h] >= 0.5 * Wmax) {", "if (hyp_W[h] >= 0.4 * Wmax) {"),
    ("pre-selection threshold", "wstar[k] >= 0.5) ? 1 : 0;", "wstar[k] >= 0.4) ? 1 : 0;"),
    ("w* last instead of max", "if (wkeep[h][k] > wstar[k]) wstar[k] = wkeep[h][k];", "wstar[k] = wkeep[h][k];"),
    # association and weights (Sec. 2)
    ("projection truncates", "double ur = floor(uf + 0.5), vr = floor(vf + 0.5);", "double ur = floor(uf), vr = floor(vf);"),
    ("tukey not squared", "om = (1.0 - t * t) * (1.0 - t * t);", "om = (1.0 - t * t);"),
    ("feature ramp 3H", "double wk = 1.0 - dk / (5.0 * s->P.H);", "double wk = 1.0 - dk / (3.0 * s->P.H);"),
    ("pre-selected weight one", "a->orbw[k] = s->wstar[k];", "a->orbw[k] = 1.0;"),
    ("dynamic arap weight without w_orb", "double sd = sumw + s->P.w_orb * sumo;", "double sd = sumw + sumo;"),
    ("zbuffer tie rule", "if (z < a->zmin[pix]) { a->zmin[pix] = z; a->zwin[pix] = j; }",
     "if (z <= a->zmin[pix]) { a->zmin[pix] = z; a->zwin[pix] = j; }"),
    # residuals and normal equations (Eqs. (1), (5), (6))
    ("angle residual sum", "for (int c = 0; c < 3; c++) rr[1 + c] = sa * (ah[c] - bh[c]);",
     "for (int c = 0; c < 3; c++) rr[1 + c] = sa * (ah[c] + bh[c]);"),
    ("length residual squared", "rr[0] = sl * (lb - l0);", "rr[0] = sl * (lb * lb - l0 * l0);"),
    ("rotation residual drops w", "for (int c = 0; c < 4; c++) rr[4 + c] = sr * (qa[c] - qb[c]);",
     "for (int c = 1; c < 4; c++) rr[4 + c] = sr * (qa[c] - qb[c]);"),
    ("length jacobian sign", "Jg[0 * 12 + 3 + c] = -sl * bh[c];", "Jg[0 * 12 + 3 + c] = sl * bh[c];"),
    ("rotation jacobian sign", "Jg[(4 + r4) * 12 + 6 + c] = -sr * 0.5 * Gb[r4 * 3 + c];",
     "Jg[(4 + r4) * 12 + 6 + c] = sr * 0.5 * Gb[r4 * 3 + c];"),
    ("angle jacobian drops projector", "Jg[(1 + r3) * 12 + 3 + c] = sa * Pbc / lb;",
     "Jg[(1 + r3) * 12 + 3 + c] = sa * ((r3 == c) ? 1.0 : 0.0) / lb;"),
    ("data jacobian drops blend weight", "Jg[rr * 6 * nb + 6 * slot_blk[t] + c] += sw * sg[t] * al[t] * acc;",
     "Jg[rr * 6 * nb + 6 * slot_blk[t] + c] += sw * sg[t] * acc;"),
    ("gradient sign", "g[cx] += Jr[x] * rg[row];", "g[cx] -= Jr[x] * rg[row];"),
    ("icp residual drops weight", "r[j] = sw * (nn[0] * (v[0] - q[0])",
     "r[j] = (nn[0] * (v[0] - q[0])"),
    # solve and LM (Sec. 2)
    ("levenberg instead of marquardt", "A[(size_t)i * n + i] = A[(size_t)i * n + i] * (1.0 + lambda) + 1e-12 * dmax;",
     "A[(size_t)i * n + i] = A[(size_t)i * n + i] + lambda + 1e-12 * dmax;"),
    ("accept within 0.1 percent", "accept = e_new < e_old;", "accept = e_new <= 1.001 * e_old;"),
    ("reject multiplies by 5", "lambda = lambda * 10.0;", "lambda = lambda * 5.0;"),
    ("accept divides by 5", "lambda = lambda / 10.0;", "lambda = lambda / 5.0;"),
    ("lower damping clamp", "if (lambda < 1e-10) lambda = 1e-10;", "if (lambda < 1e-12) lambda = 1e-12;"),
    ("arap weight every iteration", "associate(s, s->dq, &a, t == 0);\n    if (t == 0) w_arap = a.w_arap;",
     "associate(s, s->dq, &a, 1);\n    w_arap = a.w_arap;"),
    ("cholesky short inner sum", "for (int k = 0; k < j; k++) sum -= L[(size_t)i * n + k] * L[(size_t)j * n + k];",
     "for (int k = 0; k + 1 < j; k++) sum -= L[(size_t)i * n + k] * L[(size_t)j * n + k];"),
    ("back substitution transposed", "for (int k = i + 1; k < n; k++) sum -= L[(size_t)k * n + i] * x[k];",
     "for (int k = i + 1; k < n; k++) sum -= L[(size_t)i * n + k] * x[k];"),
    ("per-node solve wrong block", "B[6 * r + c] = A[(size_t)(6 * i + r) * n + 6 * i + c];",
     "B[6 * r + c] = A[(size_t)(6 * i + r) * n + c];"),
    # uniform ORB front end (Sec. 2.1)
    ("fast run of 8", "if (best < 9) return 0;", "if (best < 8) return 0;"),
    ("fast threshold not strict", "if (x > c + t) { cls[k] = 1; sb += x - c - t; }",
     "if (x >= c + t) { cls[k] = 1; sb += x - c - t; }"),
    ("suppression tie to the higher index", "if (R[q] > Ri || (R[q] == Ri && q < i)) { keep = 0; break; }",
     "if (R[q] > Ri || (R[q] == Ri && q > i)) { keep = 0; break; }"),
    ("orientation bin truncates", "int bin = (int)floor(th * 30.0 / (2.0 * ORB_PI) + 0.5);",
     "int bin = (int)floor(th * 30.0 / (2.0 * ORB_PI));"),
    ("descriptor test reversed", "if (sa < sb) d[k >> 3] |= (uint8_t)(1u << (k & 7));",
     "if (sa > sb) d[k >> 3] |= (uint8_t)(1u << (k & 7));"),
    ("pattern rotation sign", "rot[b][k][2 * h] = (int)lround(x * cs - y * sn);",
     "rot[b][k][2 * h] = (int)lround(x * cs + y * sn);"),
    ("box sum 5x3", "for (int dx = -2; dx <= 2; dx++) acc += img", "for (int dx = -1; dx <= 1; dx++) acc += img"),
    # closest-point association (the kd-tree alternative of Sec. 2)
    ("closest point ignores normal validity", "    if (!s->nvalid[p]) continue;\n    const double* q = s->qpts + 3 * p;",
     "    const double* q = s->qpts + 3 * p;"),
    ("closest point drops z", "double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];",
     "double d2 = d[0] * d[0] + d[1] * d[1];"),
]


def _build(text, out_dir, name):
    c = os.path.join(out_dir, name + ".c")
    so = os.path.join(out_dir, name + ".so")
    with open(c, "w") as f:
        f.write(text)
    r = subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-I",
                        os.path.join(ROOT, "oracle"), "-o", so, c, "-lm"], capture_output=True, text=True)
    return so if r.returncode == 0 else None


def _pins_pass(so):
    env = dict(os.environ, TT_ORACLE_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", PINS, "-x", "-q", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode == 0, r.stdout[-2000:]


def test_mutants_are_well_formed():
    with open(SRC) as f:
        src = f.read()
    names = [m[0] for m in MUTANTS]
    assert len(set(names)) == len(names)
    for name, old, new in MUTANTS:
        assert src.count(old) == 1, name
        assert old != new, name


def test_every_planted_mistake_fails_a_pin(tmp_path):
    with open(SRC) as f:
        src = f.read()
    out = str(tmp_path)
    base = _build(src, out, "unmodified")
    assert base is not None
    ok, log = _pins_pass(base)
    assert ok, "the pins fail on an unmodified copy of the oracle:\n" + log

    def run(i):
        name, old, new = MUTANTS[i]
        so = _build(src.replace(old, new), out, f"m{i:02d}")
        if so is None:
            return name, "does not compile"
        passed, _ = _pins_pass(so)
        return name, "survived" if passed else "caught"

    workers = max(1, min(8, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(run, range(len(MUTANTS))))
    bad = [(n, st) for n, st in results if st != "caught"]
    assert not bad, bad
    assert len(results) == len(MUTANTS)


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-q"]))
