"""Build libharpia.so (HIP for gfx950) from csrc/.

Every source is compiled as HIP with hipcc for --offload-arch=gfx950, in
parallel, into _build/; the objects are linked into a shared library next to
this file.  Packed FP32 instructions are disabled for all device code.  The
per-kernel resource report of the compiler is scanned and the build fails if
any kernel spills to scratch memory (the streaming kernels rely on their
register rings staying in registers).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libharpia.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = ["-x", "hip", "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-Wno-unused-function", "-I" + INCLUDE, "-I" + CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Rpass-analysis=kernel-resource-usage"]

_SCRATCH = re.compile(r"ScratchSize \[bytes/lane\]: (\d+)")
_NAME = re.compile(r"Function Name: (\S+)")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


_INC = re.compile(r'^\s*#\s*include\s+"([^"]+)"', re.M)


def _deps(path, seen=None):
    """The file and every quoted include it pulls in, transitively."""
    seen = set() if seen is None else seen
    if path in seen:
        return seen
    seen.add(path)
    for name in _INC.findall(open(path).read()):
        for d in (os.path.dirname(path), CSRC, INCLUDE):
            cand = os.path.join(d, name)
            if os.path.exists(cand):
                _deps(cand, seen)
                break
    return seen


def _headers_mtime(src):
    return max(os.path.getmtime(h) for h in _deps(src))


def _compile(src: str, force: bool):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    log = obj + ".log"
    if (not force and os.path.exists(obj)
            and os.path.getmtime(obj) >= _headers_mtime(src)):
        return obj, open(log).read() if os.path.exists(log) else ""
    cmd = [HIPCC] + CFLAGS + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    with open(log, "w") as f:
        f.write(p.stdout)
    if p.returncode != 0:
        msg = "\n".join(l for l in p.stdout.splitlines() if "remark" not in l)
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, msg[-6000:]))
    return obj, p.stdout


def _check_scratch(name: str, log: str):
    bad = []
    current = None
    for line in log.splitlines():
        m = _NAME.search(line)
        if m:
            current = m.group(1)
            continue
        m = _SCRATCH.search(line)
        if m and int(m.group(1)) > 0:
            bad.append((current, int(m.group(1))))
    if bad:
        raise RuntimeError("kernels in %s spill to scratch: %s" % (name, bad[:5]))


def build(force: bool = True, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, force), srcs))
    for src, (obj, log) in zip(srcs, results):
        _check_scratch(os.path.basename(src), log)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout[-4000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv)
    print(LIB)
