"""Compile the HIP sources of the ACE library for gfx950 into an in-tree shared library."""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libace_hip.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off: plain FP32 code must not be fused into v_pk_* forms
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


NOISE = "'-packed-fp32-ops' is not a recognized feature for this target"
# The compiler's per-kernel resource report (registers, scratch, occupancy).
RESOURCE_REMARK = "-Rpass-analysis=kernel-resource-usage"


def _run(cmd, verbose):
    """Run one hipcc command; return its kernel resource remarks as {kernel: {field: value}}."""
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    usage, name, other = {}, None, []
    for line in r.stderr.splitlines():
        if NOISE in line:
            continue
        if "kernel-resource-usage" not in line:
            other.append(line)
            continue
        text = line.split("remark:", 1)[-1].split("[-Rpass", 1)[0].strip()
        if text.startswith("Function Name:"):
            name = text.split(":", 1)[1].strip()
            usage[name] = {}
        elif name and ":" in text:
            key, val = text.rsplit(":", 1)
            usage[name][key.strip()] = val.strip()
    err = "\n".join(l for l in other if not l.lstrip().startswith(("|", "^")) and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)
    return usage


def check_resources(usage: dict, path: str) -> None:
    """Write the per-kernel report and refuse kernels that spill to scratch memory: every
    kernel here is laid out to keep its working set in registers and LDS, so a spill is a
    regression (usually a register-budget overrun after a change)."""
    bad = []
    with open(path, "w") as f:
        for name in sorted(usage):
            u = usage[name]
            f.write(f"{name}: " + ", ".join(f"{k} {v}" for k, v in u.items()) + "\n")
            if u.get("ScratchSize [bytes/lane]", "0") != "0" or u.get("VGPRs Spill", "0") != "0":
                bad.append(name)
    if bad:
        raise RuntimeError("kernels spill to scratch memory (see " + path + "):\n  " + "\n  ".join(bad))


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link the shared library."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"] + [RESOURCE_REMARK]
    jobs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        jobs.append((obj, [hipcc, *compile_flags, *inc, "-c", "-o", obj, src]))
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        reports = list(ex.map(lambda j: _run(j[1], verbose), jobs))
    usage = {}
    for rep in reports:
        usage.update(rep)
    check_resources(usage, os.path.join(objdir, "kernel_resources.txt"))
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *[j[0] for j in jobs]], verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
