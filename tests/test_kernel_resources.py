"""Resource use of every kernel in the built library, read from the AMDGPU
code-object metadata of liblbm.so (no GPU needed).

Every kernel must run without scratch memory: no private segment (register
spills to memory, or stack objects).  The populations of a cell live in
registers for the whole update (95 of them for D3Q95), so a spill would put
loads and stores to scratch on the hot path.  (A kernel that may hold more
than 256 registers per lane can spill vector registers into the accumulation
registers instead; that is a register move, not memory, and is allowed.)
"""
import os
import re
import struct
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1303_4624_amd", "liblbm.so")
READELF = "/opt/rocm/llvm/bin/llvm-readelf"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _section(path, name):
    """Bytes of ELF section `name` of a 64-bit little-endian ELF file."""
    with open(path, "rb") as fh:
        data = fh.read()
    shoff, = struct.unpack_from("<Q", data, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", data, 0x3A)
    hdr = lambda i: struct.unpack_from("<IIQQQQIIQQ", data, shoff + i * shentsize)
    stroff = hdr(shstrndx)[4]
    for i in range(shnum):
        h = hdr(i)
        nm = data[stroff + h[0]: data.index(b"\0", stroff + h[0])].decode()
        if nm == name:
            return data[h[4]: h[4] + h[5]]
    raise KeyError(name)


def _device_objects(fatbin):
    """The gfx950 code objects of every offload bundle in the section."""
    out = []
    pos = fatbin.find(MAGIC)
    while pos >= 0:
        n, = struct.unpack_from("<Q", fatbin, pos + len(MAGIC))
        p = pos + len(MAGIC) + 8
        for _ in range(n):
            off, size, tlen = struct.unpack_from("<QQQ", fatbin, p)
            triple = fatbin[p + 24: p + 24 + tlen].decode()
            p += 24 + tlen
            if "gfx950" in triple and size:
                out.append(fatbin[pos + off: pos + off + size])
        pos = fatbin.find(MAGIC, p)
    return out


def kernel_resources():
    """{mangled kernel name: {metadata key: int}} over all code objects."""
    if not os.path.exists(LIB):
        pytest.skip("liblbm.so is not built")
    if not os.path.exists(READELF):
        pytest.skip("llvm-readelf not found")
    res = {}
    for k, co in enumerate(_device_objects(_section(LIB, ".hip_fatbin"))):
        path = os.path.join("/tmp", f"lbm_co_{os.getpid()}_{k}.co")
        with open(path, "wb") as fh:
            fh.write(co)
        try:
            notes = subprocess.run([READELF, "--notes", path], capture_output=True, text=True,
                                   check=True).stdout
        finally:
            os.unlink(path)
        for blk in notes.split("\n  - ")[1:]:
            m = re.search(r"\.name:\s+(\S+)", blk)
            if not m or ".kd" in m.group(1):
                continue
            vals = {key: int(v) for key, v in re.findall(
                r"\.(private_segment_fixed_size|vgpr_spill_count|sgpr_spill_count|vgpr_count|"
                r"agpr_count|sgpr_count):\s+(\d+)", blk)}
            if "private_segment_fixed_size" in vals:
                res[m.group(1)] = vals
    return res


def test_every_kernel_is_found():
    res = kernel_resources()
    names = " ".join(res)
    # the update, the in-place update, the adjoint and the moments of each model
    for model in ("D2Q33", "D3Q95", "D3Q19", "D3Q15"):
        for kern in ("k_step", "k_step_aa", "k_adjoint", "k_moments", "k_init"):
            assert re.search(kern + r"INS_\d+" + model, names), (kern, model)


def test_no_kernel_uses_scratch_memory():
    res = kernel_resources()
    bad = {n: v for n, v in res.items() if v["private_segment_fixed_size"]}
    assert not bad, "\n".join(f"{n}: {v}" for n, v in sorted(bad.items()))
