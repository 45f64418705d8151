"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code only).

The oracle is rebuilt with -fsanitize=address,undefined (serial, first error aborts) and
driven in a child process, with the ASan runtime preloaded, through the paths the pins and
parity tests use: structured meshes with walls, far field and periodic sides, BGK and
Shakhov, the limiter, both predictors, the CFL ramp, explicit and implicit steps, a short
solve, the micro operator and sweep, and a hybrid quadrilateral/triangle mesh.  Any
out-of-bounds access, use after free or undefined operation ends the child with an error.
"""
import os
import subprocess
import sys

import pytest

from oracle import oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
import workloads as wl
from oracle import Oracle


def exercise(cfg, implicit=2, explicit=1):
    o = Oracle(cfg)
    f = o.get_state()
    o.set_state(f * wl.perturbation(f.shape, 3, 0.05))
    o.flux()
    o.face_moments()
    o.macro_residual()
    o.predict()
    D, Cc = o.micro_operator(0)
    o.micro_sweep(0, np.ones(o.nc))
    o.implicit_step(implicit)
    o.explicit_step(explicit)
    o.moments()
    o.cells()
    o.cell_sides()
    return o


exercise(wl.cavity(n=6, nj=5, stretch=1.5, nv=6, Kn=0.1))
exercise(dict(wl.shrink(wl.case("cavity_kn10"), ni=5, nj=4, nv=7), precision=wl.FP64, limiter=1))
exercise(dict(wl.cavity(n=5, nv=6, Kn=0.2), predictor=1, relax_sweeps=4))
exercise(wl.couette(nj=6, nv=6))
exercise(dict(wl.shrink(wl.case("cylinder_ma5"), ni=6, nj=8, nv=8), precision=wl.FP64))
exercise(wl.hybrid_cavity(n=6, nq=1, nv=6, jitter=0.15, seed=1, Kn=0.1))
h = wl.hybrid_cavity(n=6, nq=1, nv=6, jitter=0.15, seed=1, Kn=0.1)
exercise(wl.with_mesh(h, wl.renumbered(h["mesh"], 2)))
o = Oracle(wl.cavity(n=5, nv=6, Kn=0.1))
o.solve(1e-6, 30)
print("OK")
"""


def test_oracle_runs_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime for gcc here")
    lib = orc.build_sanitized(str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ, LD_PRELOAD=asan, IDUGKS_ORACLE_LIB=lib, OMP_NUM_THREADS="1",
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", SCRIPT], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
