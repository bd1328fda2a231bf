"""Builds libdsr.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libdsr.so")
SOURCES = [os.path.join(CSRC, "dsr_kernels.hip"), os.path.join(CSRC, "dsr_api.cpp")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-ffp-contract=off", "-fno-fast-math",
         # no packed fp32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


RESOURCES = os.path.join(PKG, "libdsr.resources.txt")


def sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in SOURCES + [os.path.join(CSRC, "dsr_internal.h"), os.path.join(ROOT, "include", "dsr_device.h"),
                        os.path.join(ROOT, "include", "dsr.h")]:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def build(verbose=False):
    """Compile every source (always) and replace libdsr.so atomically; the
    compiler's per-kernel resource remarks go to libdsr.resources.txt."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-Rpass-analysis=kernel-resource-usage", "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise subprocess.CalledProcessError(p.returncode, cmd, p.stdout, p.stderr)
    os.replace(tmp, LIB)
    with open(RESOURCES, "w") as fh:
        fh.write("sources_sha256: %s\n" % sources_hash())
        fh.write("\n".join(l for l in p.stderr.splitlines() if "remark" in l))
    return LIB


def kernel_resources():
    """Registers, scratch and occupancy of every region-kernel instance, from
    the compiler's resource remarks (a device-only compile; writes nothing
    in the tree).  Returns {instance name: {"vgprs", "scratch", "waves_per_simd"}}."""
    import re
    import tempfile
    out = None
    if os.path.exists(RESOURCES):
        with open(RESOURCES) as fh:
            text = fh.read()
        if text.startswith("sources_sha256: %s" % sources_hash()):
            out = text
    if out is None:
        with tempfile.TemporaryDirectory() as tmp:
            cmd = [HIPCC] + [f for f in FLAGS if f not in ("-shared", "-fPIC")] + [
                "-c", "--offload-device-only", "-Rpass-analysis=kernel-resource-usage",
                "-o", os.path.join(tmp, "k.o"), SOURCES[0]]
            out = subprocess.run(cmd, capture_output=True, text=True, check=True).stderr
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
