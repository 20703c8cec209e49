"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code only): a copy
built with both, loaded into a child Python with the ASan runtime preloaded, steps the mesh
kinds and boundary conditions the tests use (box and tetrahedral cells; specular, diffuse,
far-field and periodic faces; second order).  Any out-of-bounds access or undefined
behaviour aborts the child."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _libasan():
    gcc = shutil.which("gcc")
    if not gcc:
        return None
    p = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(_libasan() is None, reason="gcc with the ASan runtime is needed")
def test_oracle_steps_clean_under_asan_and_ubsan(tmp_path):
    lib = tmp_path / "liboracle.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", str(lib),
                    os.path.join(ROOT, "oracle", "ugkwp_oracle.c"), "-lm"], check=True)
    script = tmp_path / "run.py"
    script.write_text(textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {ROOT!r})
        import oracle
        oracle.LIB = {str(lib)!r}
        oracle.build = lambda force=True: oracle.LIB
        from paper_2007_13091_amd import workloads as wl
        ws = [wl.periodic_box(n=(3, 3, 2), n_ref=30),
              wl.cavity(n=4, n_ref=40),
              wl.closed_box(n=(3, 2, 2), n_ref=30, kn=2.0, bc=wl.BC_DIFFUSE, tets=True, jitter=0.1),
              wl.free_stream_box(n=(3, 3, 2), n_ref=30, kn=0.1, perturb=0.2, tets=True, jitter=0.1),
              wl.sod(nx=8, ny=1, nz=1, n_ref=30)]
        for w in ws:
            o = oracle.Oracle(w.mesh, w.params)
            o.set_state(w.W0)
            for _ in range(3):
                o.step()
        w = wl.sod(nx=8, ny=1, nz=1, n_ref=30)
        w.params.recon = 2
        o = oracle.Oracle(w.mesh, w.params)
        o.set_state(w.W0)
        o.step()
        o.step()
        print("sanitized run complete", flush=True)
    """))
    # the ASan runtime must come first; whatever the environment already preloads stays after it
    pre = ":".join(p for p in (_libasan(), os.environ.get("LD_PRELOAD", "")) if p)
    env = dict(os.environ, LD_PRELOAD=pre, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized run complete" in r.stdout
