"""Builds libdsr.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

The region kernel is compiled once per instance listed in DSR_INSTANCES
(csrc/dsr_internal.h), each in its own hipcc process, in parallel; the
host-only sources are compiled beside them and everything is linked into
one shared library."""
import os
import re
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libdsr.so")
KERNEL = os.path.join(CSRC, "dsr_kernels.hip")
HOST_SOURCES = [os.path.join(CSRC, "dsr_api.cpp"), os.path.join(CSRC, "dsr_dispatch.cpp"),
                os.path.join(CSRC, "dsr_static.hip"), os.path.join(CSRC, "dsr_ceiling.hip")]
SOURCES = [KERNEL] + HOST_SOURCES
HEADERS = [os.path.join(CSRC, "dsr_internal.h"), os.path.join(ROOT, "include", "dsr_device.h"),
           os.path.join(ROOT, "include", "dsr.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-ffp-contract=off", "-fno-fast-math",
         # no packed fp32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


RESOURCES = os.path.join(PKG, "libdsr.resources.txt")


def instances():
    """(tag, max workgroup, variant) of every compiled kernel instance."""
    with open(os.path.join(CSRC, "dsr_internal.h")) as fh:
        text = fh.read()
    body = text[text.index("#define DSR_INSTANCES(X)"):]
    body = body[:body.index("\n\n")]
    return [(t, int(w), int(v)) for t, w, v in re.findall(r"X\((\w+),\s*(\d+),\s*(-?\d+)\)", body)]


def sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in SOURCES + HEADERS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise subprocess.CalledProcessError(p.returncode, cmd, p.stdout, p.stderr)
    return p.stderr


def build(verbose=False, jobs=None):
    """Compile every source (always) and replace libdsr.so atomically; the
    compiler's per-kernel resource remarks go to libdsr.resources.txt."""
    jobs = jobs or min(8, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory() as tmp:
        cmds = []
        for tag, maxwg, variant in instances():
            cmds.append([HIPCC] + FLAGS + ["-DDSR_INST_MAXWG=%d" % maxwg, "-DDSR_INST_VARIANT=%d" % variant,
                                           "-DDSR_INST_TAG=%s" % tag, "-Rpass-analysis=kernel-resource-usage",
                                           "-c", "-o", os.path.join(tmp, "k_%s.o" % tag), KERNEL])
        for src in HOST_SOURCES:
            cmds.append([HIPCC] + FLAGS + ["-c", "-o", os.path.join(tmp, os.path.basename(src) + ".o"), src])
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(jobs) as ex:
            logs = list(ex.map(_run, cmds))
        objs = [c[c.index("-o") + 1] for c in cmds]
        tmp_lib = LIB + ".tmp%d" % os.getpid()
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_lib] + objs)
    os.replace(tmp_lib, LIB)
    with open(RESOURCES, "w") as fh:
        fh.write("sources_sha256: %s\n" % sources_hash())
        fh.write("\n".join(l for log in logs for l in log.splitlines() if "remark" in l))
    return LIB


def kernel_resources():
    """Registers, scratch and occupancy of every region-kernel instance, from
    the compiler's resource remarks (a device-only compile; writes nothing
    in the tree).  Returns {instance name: {"vgprs", "scratch", "waves_per_simd"}}."""
    out = None
    if os.path.exists(RESOURCES):
        with open(RESOURCES) as fh:
            text = fh.read()
        if text.startswith("sources_sha256: %s" % sources_hash()):
            out = text
    if out is None:
        with tempfile.TemporaryDirectory() as tmp:
            cmds = [[HIPCC] + [f for f in FLAGS if f != "-fPIC"] + [
                "-DDSR_INST_MAXWG=%d" % w, "-DDSR_INST_VARIANT=%d" % v, "-DDSR_INST_TAG=%s" % t,
                "-c", "--offload-device-only", "-Rpass-analysis=kernel-resource-usage",
                "-o", os.path.join(tmp, "k_%s.o" % t), KERNEL] for t, w, v in instances()]
            with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
                out = "\n".join(ex.map(_run, cmds))
    res, cur = {}, None
    for line in out.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            res[cur] = {}
            continue
        for key, pat in (("vgprs", r"\bVGPRs: (\d+)"), ("scratch", r"ScratchSize \[bytes/lane\]: (\d+)"),
                         ("waves_per_simd", r"Occupancy \[waves/SIMD\]: (\d+)")):
            m = re.search(pat, line)
            if m and cur:
                res[cur][key] = int(m.group(1))
    return res


if __name__ == "__main__":
    print(build(verbose=True))
