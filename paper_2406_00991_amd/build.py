"""Build the HIP library libpmgw.so in-tree for gfx950 (hipcc, no JIT cache).

After compiling, the device code is also compiled to AMD assembly and checked: the build fails if
any function contains a long-branch sequence (s_getpc/s_add/s_setpc to a label). In non-entry
functions the compiler's long-branch expansion has been seen to use s[30:31], the register that
holds the function's return address, which makes the function return into its own body. Keeping
every function within the short-branch range rules that out.
"""
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "pmgw.hip")
LIB = os.path.join(HERE, "libpmgw.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _asm_cmd(asm):
    return [_hipcc(), *FLAGS, "--cuda-device-only", "-S", SRC, "-o", asm]


def check_device_asm(verbose=False, asm_text=None):
    """Compile the device code to assembly (unless given); return per-kernel resource usage.
    Raises on long branches."""
    if asm_text is None:
        with tempfile.TemporaryDirectory() as td:
            asm = os.path.join(td, "dev.s")
            subprocess.run(_asm_cmd(asm), check=True, stderr=subprocess.DEVNULL)
            asm_text = open(asm).read()
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


def build(verbose=False, check=True):
    """Compile the library and (concurrently) the device assembly for the check."""
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), *FLAGS, "-fPIC", "-shared", SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    with tempfile.TemporaryDirectory() as td:
        asm = os.path.join(td, "dev.s")
        chk = subprocess.Popen(_asm_cmd(asm), stderr=subprocess.DEVNULL) if check else None
        lib = subprocess.Popen(cmd)
        rc_lib = lib.wait()
        rc_chk = chk.wait() if chk else 0
        if rc_lib != 0:
            raise subprocess.CalledProcessError(rc_lib, cmd)
        if rc_chk != 0:
            raise subprocess.CalledProcessError(rc_chk, _asm_cmd(asm))
        if check:
            check_device_asm(verbose, open(asm).read())
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, check="--no-check" not in sys.argv)
    print(LIB)
