"""Build the HIP library libpmgw.so in-tree for gfx950 (hipcc, no JIT cache).

The library is compiled as several translation units in parallel: the host API (pmgw.hip), the
solve kernels once per V-cycle precision and direction (pmgw_solve.hip), and the Runge-Kutta
stage kernels and their adjoints (pmgw_stage.hip); the objects are linked into one shared
library.

Every compile keeps its device assembly (-save-temps), and the build checks it: it fails if any
function contains a long-branch sequence (s_getpc/s_add/s_setpc to a label). In non-entry
functions the compiler's long-branch expansion has been seen to use s[30:31], the register that
holds the function's return address, which makes the function return into its own body. Keeping
every function within the short-branch range rules that out.
"""
import glob
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpmgw.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

# (source, extra defines) of each translation unit
UNITS = [
    ("pmgw.hip", []),
    ("pmgw_solve.hip", ["-DPMGW_TV=float", "-DPMGW_TR=0", "-DPMGW_TV_IS_FLOAT"]),
    ("pmgw_solve.hip", ["-DPMGW_TV=double", "-DPMGW_TR=0"]),
    ("pmgw_solve.hip", ["-DPMGW_TV=float", "-DPMGW_TR=1"]),
    ("pmgw_solve.hip", ["-DPMGW_TV=double", "-DPMGW_TR=1"]),
    ("pmgw_solve.hip", ["-DPMGW_TV=float", "-DPMGW_TR=0", "-DPMGW_WIDE"]),
    ("pmgw_solve.hip", ["-DPMGW_TV=double", "-DPMGW_TR=0", "-DPMGW_WIDE"]),
    ("pmgw3d.hip", []),
    ("pmgw_stage.hip", ["-DPMGW_STAGE_PART=0"]),
    ("pmgw_stage.hip", ["-DPMGW_STAGE_PART=1"]),
]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def check_device_asm(verbose=False, asm_text=None):
    """Per-kernel resource usage from device assembly text. Raises on long branches."""
    text = asm_text
    if ".Lpost_getpc" in text:
        raise RuntimeError("device code contains long-branch sequences (s_getpc/s_setpc); "
                           "split or shrink the offending function")
    stats = {}
    for blk in re.finditer(r"\.name:\s+(\S+)(.*?)(?=\n\s+- |\Z)", text, re.S):
        name, body = blk.group(1), blk.group(2)
        get = lambda key: int(re.search(rf"\.{key}:\s+(\d+)", body).group(1)) \
            if re.search(rf"\.{key}:\s+(\d+)", body) else None
        stats[name] = dict(vgpr=get("vgpr_count"), spill=get("vgpr_spill_count"),
                           scratch=get("private_segment_fixed_size"),
                           lds=get("group_segment_fixed_size"))
    if verbose:
        for k, v in sorted(stats.items()):
            print(f"  {k[:70]:70s} {v}")
    return stats


def build(verbose=False, check=True, jobs=None):
    """Compile every translation unit in parallel (at most `jobs` at once), check the device
    assembly, link. Returns the library path."""
    jobs = jobs or min(len(UNITS), max(1, os.cpu_count() or 1), 16)
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory() as td:
        procs, objs, dirs = [], [], []
        pending = list(enumerate(UNITS))
        running = []
        while pending or running:
            while pending and len(running) < jobs:
                i, (src, defs) = pending.pop(0)
                wd = os.path.join(td, f"u{i}")
                os.makedirs(wd)
                obj = os.path.join(wd, f"u{i}.o")
                cmd = [_hipcc(), *FLAGS, *defs, "-fPIC", "-c"]
                if check:
                    cmd.append("-save-temps")
                cmd += [os.path.join(CSRC, src), "-o", obj]
                if verbose:
                    print(" ".join(cmd), flush=True)
                running.append((cmd, subprocess.Popen(cmd, cwd=wd, stderr=subprocess.PIPE)))
                objs.append(obj)
                dirs.append(wd)
            cmd, pr = running.pop(0)
            _, err = pr.communicate()
            if pr.returncode != 0:
                for _, q in running:
                    q.kill()
                sys.stderr.write(err.decode(errors="replace"))
                raise subprocess.CalledProcessError(pr.returncode, cmd)
        if check:
            text = ""
            for wd in dirs:
                for s in glob.glob(os.path.join(wd, "*amdgcn-amd-amdhsa*gfx950*.s")):
                    text += open(s).read()
            if not text:
                raise RuntimeError("no device assembly found for the long-branch check")
            check_device_asm(verbose, text)
        link = [_hipcc(), *FLAGS, "-fPIC", "-shared", *objs, "-o", tmp]
        lk = subprocess.run(link, stderr=subprocess.PIPE)
        if lk.returncode != 0:
            sys.stderr.write(lk.stderr.decode(errors="replace"))
            raise subprocess.CalledProcessError(lk.returncode, link)
    os.replace(tmp, LIB)
    return LIB


def device_stats(verbose=True):
    """Build with the assembly kept and print per-kernel VGPR / spill / scratch / LDS use."""
    stats = {}
    with tempfile.TemporaryDirectory() as td:
        for i, (src, defs) in enumerate(UNITS):
            asm = os.path.join(td, f"u{i}.s")
            subprocess.run([_hipcc(), *FLAGS, *defs, "--cuda-device-only", "-S",
                            os.path.join(CSRC, src), "-o", asm], check=True,
                           stderr=subprocess.DEVNULL)
            stats.update(check_device_asm(False, open(asm).read()))
    if verbose:
        for k, v in sorted(stats.items()):
            print(f"  {k[:70]:70s} {v}")
    return stats


if __name__ == "__main__":
    if "--stats" in sys.argv:
        device_stats()
    else:
        build(verbose="-v" in sys.argv, check="--no-check" not in sys.argv)
        print(LIB)
