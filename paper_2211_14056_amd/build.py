"""Build step: emit the generated matrix-element code and compile libmfhip.so for gfx950.

Usage: python -m paper_2211_14056_amd.build [--jobs N]
"""
import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
GEN = os.path.join(CSRC, 'generated')
OUT = os.path.join(HERE, 'libmfhip.so')
BUILD = os.path.join(HERE, '_build')

SOURCES = ['me_vjp_ttgg_f64.hip', 'me_vjp_ttgg_f32.hip', 'me_batch_f64.hip', 'me_batch_mfma.hip', 'me_batch_f32.hip',
           'me_vjp_small.hip', 'me_kernels.hip', 'me_mfma.hip', 'mf_api.cpp', 'phase_space.hip', 'me_vjp.hip',
           'me_batch.hip', 'vegas.hip', 'me_ttgg_quad.hip', 'me_ttgg_pair.hip', 'unweight.hip', 'hadronic.hip', 'me_bg.hip',
           'me_quark.hip']

FLAGS = ['--offload-arch=gfx950', '-O3', '-std=c++17', '-fPIC', '-ffp-contract=fast',
         # no packed FP32 arithmetic anywhere in device code
         '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
         '-Wno-unused-command-line-argument']


def hipcc():
    for c in ('/opt/rocm/bin/hipcc', shutil.which('hipcc') or ''):
        if c and os.path.exists(c):
            return c
    raise RuntimeError('hipcc not found')


def generate():
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2211_14056_amd.gen import process_compiler
    return process_compiler.emit_all(GEN)


def _deps(obj):
    """Files the object was compiled from, from the dependency file the compiler wrote (None if absent)."""
    d = obj[:-2] + '.d'
    if not os.path.exists(d):
        return None
    text = open(d).read().replace('\\\n', ' ')
    out = []
    for line in text.splitlines():
        if ':' in line:
            out += line.split(':', 1)[1].split()
    return out


def _up_to_date(obj):
    if not os.path.exists(obj):
        return False
    deps = _deps(obj)
    if deps is None:
        return False
    t = os.path.getmtime(obj)
    return all(os.path.exists(f) and os.path.getmtime(f) <= t for f in deps)


def compile_one(src, extra=(), incremental=False):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + '.o')
    if incremental and _up_to_date(obj):
        return obj
    cmd = [hipcc()] + FLAGS + list(extra) + ['-MMD', '-MF', obj[:-2] + '.d', '-c', os.path.join(CSRC, src),
                                               '-o', obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f'compile failed: {src}\n{r.stderr[-4000:]}')
    return obj


def build(jobs=None, verbose=True, incremental=False):
    """Generate and compile everything (incremental=True skips up-to-date objects)."""
    os.makedirs(BUILD, exist_ok=True)
    if incremental and os.path.isdir(GEN):
        # regenerate into a scratch copy; keep file times when the text is unchanged
        import filecmp
        import tempfile
        tmp = tempfile.mkdtemp()
        sys.path.insert(0, os.path.dirname(HERE))
        from paper_2211_14056_amd.gen import process_compiler
        process_compiler.emit_all(tmp)
        for f in os.listdir(tmp):
            dst = os.path.join(GEN, f)
            if not (os.path.exists(dst) and filecmp.cmp(os.path.join(tmp, f), dst, shallow=False)):
                shutil.copy(os.path.join(tmp, f), dst)
        shutil.rmtree(tmp)
    else:
        generate()
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: compile_one(s, incremental=incremental), srcs))
    tmp = OUT + '.tmp'
    cmd = [hipcc(), '--offload-arch=gfx950', '-shared', '-fPIC'] + objs + ['-o', tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f'link failed\n{r.stderr[-4000:]}')
    os.replace(tmp, OUT)
    if verbose:
        print(f'built {OUT}')
    return OUT


if __name__ == '__main__':
    ap = argparse.ArgumentParser()
    ap.add_argument('--jobs', type=int, default=None)
    ap.add_argument('--incremental', action='store_true')
    args = ap.parse_args()
    build(args.jobs, incremental=args.incremental)
