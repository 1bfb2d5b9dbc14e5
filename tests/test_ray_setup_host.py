"""The raymarcher's per-ray geometry (double-float FP32, render_dev.hpp) against the FP64 definition,
on the CPU: the device functions are compiled for the host with g++ (the hardware reciprocal and
square root replaced by correctly rounded ones moved by -1, 0 or +1 ulp at random, which covers the
hardware's one-ulp approximations) next to a plain FP64 statement of the geometry (Sec. 2.4: pixel
centre ray, slab clip against [0, (n-1) h], N = ceil(L / delta) segments of delta = step min h, the
last one shorter, samples at the segment midpoints), for orthographic and perspective cameras, axis-
aligned ones among them (exact integer chord ratios), anisotropic grids and several steps.  N must
agree exactly, and the 32.32 fixed-point positions and steps within one unit of 2^-32 voxel."""
import re
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2605_19737_amd" / "csrc"

HARNESS = r"""
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#define __device__
#define __forceinline__ inline
static std::mt19937 prng(11);
static float nudge(float x)
{
    const int k = (int)(prng() % 3u) - 1;
    return k < 0 ? std::nextafterf(x, -INFINITY) : (k > 0 ? std::nextafterf(x, INFINITY) : x);
}
static float __builtin_amdgcn_rcpf(float x) { return nudge(1.0f / x); }
static float __builtin_amdgcn_sqrtf(float x) { return nudge(std::sqrt(x)); }
@STRUCTS@
@HELPERS@
@DEVICE@

// the FP64 definition
struct Ref { long long N; long long q0[3], ql[3], dq[3]; double delta, dlast; };
static long long fix64(double q, int n)
{
    double v = q * 4294967296.0;
    const double hi = (double)(n - 1) * 4294967296.0 - 1.0;
    v = v < 0.0 ? 0.0 : (v > hi ? hi : v);
    return llrint(v);
}
static Ref ref_ray(const KCam &c, int pi, int pj, const int n[3], const float h[3], float step)
{
    Ref r; r.N = 0;
    const double fi = pi + 0.5, fj = pj + 0.5;
    double o[3], d[3];
    if (c.persp) {
        double n2 = 0.0;
        for (int a = 0; a < 3; ++a) { o[a] = c.o[a]; d[a] = (double)c.d0[a] + fi * c.du[a] + fj * c.dv[a]; n2 += d[a] * d[a]; }
        const double nn = std::sqrt(n2);
        for (int a = 0; a < 3; ++a) d[a] /= nn;
    } else {
        for (int a = 0; a < 3; ++a) { o[a] = (double)c.o[a] + fi * c.du[a] + fj * c.dv[a]; d[a] = c.d0[a]; }
    }
    double t0 = -INFINITY, t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        const double hi = (double)(n[a] - 1) * h[a];
        if (d[a] == 0.0) { if (o[a] < 0.0 || o[a] > hi) return r; continue; }
        double ta = -o[a] / d[a], tb = (hi - o[a]) / d[a];
        if (ta > tb) std::swap(ta, tb);
        t0 = std::max(t0, ta);
        t1 = std::min(t1, tb);
    }
    const double tn = t0 > 0.0 ? t0 : 0.0, tf = t1;
    if (!(tf > tn)) return r;
    const double delta = (double)step * std::min(h[0], std::min(h[1], h[2]));
    const double L = tf - tn;
    const long long N = (long long)std::ceil(L / delta);
    const double dlast = L - (double)(N - 1) * delta;
    const double tfirst = tn + 0.5 * (N == 1 ? dlast : delta), tlast = tn + (double)(N - 1) * delta + 0.5 * dlast;
    for (int a = 0; a < 3; ++a) {
        r.q0[a] = fix64((o[a] + tfirst * d[a]) / h[a], n[a]);
        r.ql[a] = fix64((o[a] + tlast * d[a]) / h[a], n[a]);
        r.dq[a] = llrint(delta * d[a] / h[a] * 4294967296.0);
    }
    r.N = N; r.delta = delta; r.dlast = dlast;
    return r;
}

int main()
{
    std::mt19937 rng(7);
    std::uniform_real_distribution<float> U(-1.f, 1.f);
    long rays = 0, hits = 0, badN = 0, badq = 0, badlen = 0;
    for (int cfg = 0; cfg < 120; ++cfg) {
        int n[3] = {181, 217, 181};
        float h[3] = {1.f, 1.f, 1.f};
        if (cfg % 3 == 1) { n[0] = 96 + cfg % 50; n[1] = 130; n[2] = 40; h[0] = 0.7f; h[1] = 0.7f; h[2] = 3.3f; }
        if (cfg % 3 == 2) { n[0] = 512; n[1] = 512; n[2] = 400; h[0] = 0.45f; h[1] = 0.45f; h[2] = 0.6f; }
        const float step = (cfg % 5 == 0) ? 0.37f : 0.5f;
        KGrid g;
        for (int a = 0; a < 3; ++a) g.n[a] = n[a];
        set_grid_steps(g, h, step);
        KCam c;
        c.persp = cfg % 2;
        const float ctr[3] = {0.5f * (n[0] - 1) * h[0], 0.5f * (n[1] - 1) * h[1], 0.5f * (n[2] - 1) * h[2]};
        float ang = cfg * 0.37f, el = 0.3f * U(rng);
        if (cfg % 7 == 3) { ang = 0.f; el = 0.f; }  // axis-aligned
        const float dist = (cfg % 4 == 0) ? 1500.f : 600.f;
        const float fw[3] = {std::cos(ang) * std::cos(el), std::sin(ang) * std::cos(el), std::sin(el)};
        float rt[3] = {fw[1], -fw[0], 0.f};
        const float rn = std::sqrt(rt[0] * rt[0] + rt[1] * rt[1]);
        for (int a = 0; a < 3; ++a) rt[a] /= rn;
        const float up[3] = {rt[1] * fw[2] - rt[2] * fw[1], rt[2] * fw[0] - rt[0] * fw[2], rt[0] * fw[1] - rt[1] * fw[0]};
        const int W = 48, H = 48;
        for (int a = 0; a < 3; ++a) {
            if (c.persp) {
                const float px = 0.5f / W;
                c.o[a] = ctr[a] - dist * fw[a]; c.du[a] = px * rt[a]; c.dv[a] = -px * up[a];
                c.d0[a] = fw[a] - 0.5f * W * c.du[a] - 0.5f * H * c.dv[a];
            } else {
                c.d0[a] = fw[a]; c.du[a] = 300.f / W * rt[a]; c.dv[a] = -300.f / H * up[a];
                c.o[a] = ctr[a] - dist * fw[a] - 0.5f * W * c.du[a] - 0.5f * H * c.dv[a];
            }
        }
        for (int pj = 0; pj < H; ++pj)
            for (int pi = 0; pi < W; ++pi) {
                const RayGeo r = ray_setup(c, pi, pj, g);
                const Ref f = ref_ray(c, pi, pj, n, h, step);
                ++rays;
                if (r.N != f.N) { ++badN; continue; }
                if (!r.N) continue;
                ++hits;
                for (int a = 0; a < 3; ++a) {
                    // the last full step as the device keeps it inside the grid (same clamp as the device)
                    long long st = f.dq[a];
                    if (f.N >= 3) {
                        const long long maxq = (long long)(n[a] - 1) * 4294967296LL - 1, end = f.q0[a] + (f.N - 2) * st;
                        if (end < 0) st = (0 - f.q0[a]) / (f.N - 2);
                        else if (end > maxq) st = (maxq - f.q0[a]) / (f.N - 2);
                    }
                    const long long q0 = f.N == 1 ? f.ql[a] : f.q0[a];
                    if (llabs(r.q0[a] - q0) > 1 || llabs(r.ql[a] - f.ql[a]) > 1 || llabs(r.dq[a] - st) > 1) ++badq;
                }
                if (r.delta != (float)f.delta || std::fabs((double)r.dlast - f.dlast) > 1e-6 * f.delta) ++badlen;
            }
    }
    printf("rays %ld hits %ld badN %ld badq %ld badlen %ld\n", rays, hits, badN, badq, badlen);
    return 0;
}
"""


def _block(text, start, end):
    a = text.index(start)
    b = text.index(end, a)
    return text[a:b]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_ray_setup_matches_fp64_definition(tmp_path):
    dev = (CSRC / "render_dev.hpp").read_text()
    args = (CSRC / "render_args.hpp").read_text()
    device = _block(dev, "struct RayGeo {", "// TF in LDS")
    structs = _block(args, "struct KCam {", "struct KFeat {") + _block(args, "struct KGrid {", "struct KTF {")
    helpers = _block(args, "inline void split2(", "}  // namespace dvr")
    src = HARNESS.replace("@STRUCTS@", structs).replace("@HELPERS@", helpers).replace("@DEVICE@", device)
    (tmp_path / "rs.cpp").write_text(src)
    exe = tmp_path / "rs"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-o", str(exe), str(tmp_path / "rs.cpp")],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    print(out)
    m = dict(re.findall(r"(\w+) (\d+)", out))
    assert int(m["rays"]) == 120 * 48 * 48 and int(m["hits"]) > 100000
    assert int(m["badN"]) == 0 and int(m["badq"]) == 0 and int(m["badlen"]) == 0
