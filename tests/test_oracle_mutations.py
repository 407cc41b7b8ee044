"""Mutation check of the oracle's pins: every plausible mistake below, planted in a scratch
copy of oracle/oracle.cpp, must make at least one test of tests/test_oracle_pins.py fail.

Each mutant is compiled with the oracle's own flags into a temporary directory and the pin
suite runs against it in a child process (FLOD_ORACLE_LIB names the mutant library). The
unmutated source, built the same way, must pass the same suite, so a failure means the
pins caught the mistake and not that the harness is broken. Nothing under oracle/ is
modified.

Each mutation names the passage (or the 3DGS-framework convention the paper builds on)
whose arithmetic it breaks.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")

# (name, what it breaks, [(old, new), ...]); every `old` must occur in the source.
MUTATIONS = [
    ("sh_view_direction_flipped", "SH colour at dir = (mu - eye) (Preliminary: SH colour)",
     [("T dx = mu[0] - cam.campos[0], dy = mu[1] - cam.campos[1], dz = mu[2] - cam.campos[2];",
       "T dx = cam.campos[0] - mu[0], dy = cam.campos[1] - mu[1], dz = cam.campos[2] - mu[2];"),
      ("double dir[3] = {means[g * 3 + 0] - cam.campos[0], means[g * 3 + 1] - cam.campos[1],\n"
       "                     means[g * 3 + 2] - cam.campos[2]};",
       "double dir[3] = {cam.campos[0] - means[g * 3 + 0], cam.campos[1] - means[g * 3 + 1],\n"
       "                     cam.campos[2] - means[g * 3 + 2]};")]),
    ("fov_clamp_1_6", "EWA Jacobian clamp at 1.3x the half field of view (eq. 2's Sigma')",
     [("fov_clamp = 1.3f;", "fov_clamp = 1.6f;"), ("fov_clamp = 1.3;", "fov_clamp = 1.6;")]),
    ("no_fov_clamp", "EWA Jacobian clamp (eq. 2's Sigma')",
     [("T xc = tmin(tmax(u, -limx), limx);", "T xc = u;"), ("T yc = tmin(tmax(v, -limy), limy);", "T yc = v;")]),
    ("dilation_0_2", "0.3 px^2 dilation of Sigma'",
     [("dilate = 0.3f", "dilate = 0.2f"), ("dilate = 0.3,", "dilate = 0.2,")]),
    ("ewa_jacobian_sign", "EWA Jacobian J = d(pixel)/d(view point)",
     [("J02 = -(cam.fx * xc) / p.tz;", "J02 = (cam.fx * xc) / p.tz;")]),
    ("alpha_clamp_0_999", "alpha = min(0.99, o G) (eq. 2)", [("a_max = 0.99", "a_max = 0.999")]),
    ("alpha_skip_1_128", "skip alpha < 1/255", [("a_min = 1.0 / 255.0", "a_min = 1.0 / 128.0")]),
    ("stop_threshold_1e_3", "stop when T falls below 1e-4", [("t_min = 1e-4", "t_min = 1e-3")]),
    ("stopping_gaussian_blended", "the Gaussian that would take T below 1e-4 is not blended",
     [("if (Tn < t_min) break;", "if (T < t_min) break;")]),
    ("support_cut_16", "support cut q <= 9", [("q_cut = 9.0", "q_cut = 16.0")]),
    ("pixel_centre_corner", "pixel centres at (x + 0.5, y + 0.5)",
     [("double px = pix_xy[2 * p] + 0.5, py = pix_xy[2 * p + 1] + 0.5;",
       "double px = pix_xy[2 * p] + 0.0, py = pix_xy[2 * p + 1] + 0.0;")]),
    ("opacity_sigmoid_sign", "o = sigmoid(logit)", [("p.opac = T(1.0) / (T(1.0) + ex(-logit));",
                                                    "p.opac = T(1.0) / (T(1.0) + ex(logit));")]),
    ("scale_floor_dropped", "eq. 4: s = exp(s_opt) + s_min",
     [("s[i] = T(double((float)std::exp(val(ls[i])))) + smin;", "s[i] = T(double((float)std::exp(val(ls[i]))));"),
      ("s[i] = ex(ls[i]) + smin;", "s[i] = ex(ls[i]);")]),
    ("rotation_transposed", "eq. 1: R from the unit quaternion (w, x, y, z)",
     [("R[1] = two * (x * y - w * z);", "R[1] = two * (x * y + w * z);"),
      ("R[3] = two * (x * y + w * z);", "R[3] = two * (x * y - w * z);"),
      ("R[2] = two * (x * z + w * y);", "R[2] = two * (x * z - w * y);"),
      ("R[6] = two * (x * z - w * y);", "R[6] = two * (x * z + w * y);"),
      ("R[5] = two * (y * z - w * x);", "R[5] = two * (y * z + w * x);"),
      ("R[7] = two * (y * z + w * x);", "R[7] = two * (y * z - w * x);")]),
    ("covariance_scale_not_squared", "eq. 1: Sigma = R S S^T R^T",
     [("M[i * 3 + j] = R[i * 3 + j] * s[j];", "M[i * 3 + j] = R[i * 3 + j] * sq(s[j]);")]),
    ("conic_offdiagonal_sign", "conic = inverse of Sigma' (eq. 2)", [("p.cb = -p.b * inv;", "p.cb = p.b * inv;")]),
    ("sh_offset_dropped", "SH colour + 0.5", [("acc = acc + T(0.5);", "acc = acc;")]),
    ("sh_colour_clamp_dropped", "colour clamped at 0", [("p.rgb[ch] = p.clamped[ch] ? T(0.0) : acc;",
                                                       "p.rgb[ch] = acc;")]),
    ("sh_legendre_recursion", "real SH basis (Bonnet's recursion)",
     [("P[l + 1][j] = ((2 * l + 1) * zp - l * P[l - 1][j]) / (l + 1);",
       "P[l + 1][j] = ((2 * l) * zp - l * P[l - 1][j]) / (l + 1);")]),
    ("depth_order_descending", "alpha blending front to back in depth order",
     [("if (a.depth != b.depth) return a.depth < b.depth;", "if (a.depth != b.depth) return a.depth > b.depth;")]),
    ("tie_order_descending", "equal depths ordered by index", [("return a.idx < b.idx;", "return a.idx > b.idx;")]),
    ("near_plane_dropped", "near-plane cull at z = 0.2", [("if (!(p.tz > K<double>::near_z)) return;",
                                                          "if (!(p.tz > 0.0)) return;")]),
    ("opacity_cull_dropped", "opacity cull below 1/255", [("if (logit < logit_min) return;", "")]),
    ("footprint_ceil", "tile footprint of the support ellipse",
     [("double x1 = std::floor((mx + right) * 0.0625);", "double x1 = std::ceil((mx + right) * 0.0625);")]),
    ("band_edges_closed_above", "eq. 6: d_proj^(l-1) > d >= d_proj^(l)",
     [("keep[i] = (lo2 <= d2 && d2 < hi2) ? 1 : 0;", "keep[i] = (lo2 < d2 && d2 <= hi2) ? 1 : 0;")]),
    ("dalpha_suffix_sign", "dL/dalpha = T c - S / (1 - alpha) (backward of the blend)",
     [("dalpha += dC[ch] * (e.T * g.rgb[ch] - S[ch] / (1.0 - e.alpha));",
       "dalpha += dC[ch] * (e.T * g.rgb[ch] + S[ch] / (1.0 - e.alpha));")]),
    ("saturated_alpha_gradient", "no gradient through alpha = 0.99", [("if (!e.clamp) {", "if (true) {")]),
    ("prune_two_neighbours", "overlap pruning: mean distance to the three nearest",
     [("const double avg = ((best[0] + best[1]) + best[2]) / 3.0;", "const double avg = (best[0] + best[1]) / 2.0;")]),
    ("prune_not_strict", "overlap pruning: removal iff d_avg < d_op", [("keep[t] = (avg < d_op) ? 0 : 1;",
                                                                       "keep[t] = (avg <= d_op) ? 0 : 1;")]),
    ("transition_wrong_floor", "eq. 5: s_opt' = log(s^(l) - s_min^(l+1))",
     [("out[i] = std::log(s - s_min_next);", "out[i] = std::log(s - s_min_l);")]),
]

CXX = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC"]


def _mutate(src: str, edits) -> str:
    for old, new in edits:
        assert old in src, f"mutation anchor not found: {old!r}"
        src = src.replace(old, new)
    return src


def _build(text: str, path: str) -> None:
    cpp = path[:-3] + ".cpp"
    with open(cpp, "w") as fh:
        fh.write(text)
    subprocess.run([*CXX, "-o", path, cpp], check=True, capture_output=True)


def _run_pins(lib: str) -> subprocess.CompletedProcess:
    env = dict(os.environ, FLOD_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-m", "pytest", PINS, "-x", "-q", "-p", "no:cacheprovider",
                           "-p", "no:randomly"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_every_mutation_fails_a_pin(tmp_path):
    src = open(SRC).read()
    jobs = [("unmutated", src)] + [(name, _mutate(src, edits)) for name, _, edits in MUTATIONS]
    libs = {name: str(tmp_path / f"lib_{name}.so") for name, _ in jobs}
    workers = max(1, min(8, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda j: _build(j[1], libs[j[0]]), jobs))
    with cf.ThreadPoolExecutor(max(1, workers // 2)) as ex:
        results = dict(zip([n for n, _ in jobs], ex.map(lambda j: _run_pins(libs[j[0]]), jobs)))
    base = results.pop("unmutated")
    assert base.returncode == 0, "the unmutated oracle must pass its pins:\n" + base.stdout[-3000:]
    survived = [name for name, r in results.items() if r.returncode != 1]
    errors = {name: results[name].stdout[-1500:] for name in survived if results[name].returncode != 0}
    assert not errors, f"pin suite errored (not failed) on: {errors}"
    assert not survived, f"mutations no pin catches: {survived}"


@pytest.mark.parametrize("name,why,edits", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_anchors_exist(name, why, edits):
    src = open(SRC).read()
    for old, _ in edits:
        assert old in src, (name, old)
