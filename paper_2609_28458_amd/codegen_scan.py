"""Scan the library's device assembly for one code-generation hazard.

hipcc for gfx950 (ROCm 7.2) can place the spill of a value that leaves a
divergent region -- a store to per-lane scratch, or a copy into an
accumulation register -- in the region's join block ahead of the exec-mask
restore (``s_or_b64 exec, exec, ...``).  The spill then runs for the region's
lanes only, and the lanes that skipped the region later reload a stale value:
silently wrong results, no fault.

``scan`` reports every such spill in a join block, that is a block reached by
``s_cbranch_execz`` in which a spill comes before the block's exec restore.
A join inside a loop is a hazard: the masked-off lanes are still live there.
A join outside every loop is, in these kernels, the static-schedule start of
a persistent kernel (``if (g < n) start(g)``), whose masked-off lanes never
become live; those are reported with ``in_loop`` false.

``device_asm`` compiles every translation unit of the library to device
assembly with the flags of the library build.  Run as a module it prints the
findings and exits non-zero if a join inside a loop holds a spill.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List

from . import build

_FUNC = re.compile(r"^(_Z\w+):")
_LABEL = re.compile(r"^(\.LBB\w+):(.*)$")
_FALL = re.compile(r"^; %bb\.\d+:")
_EXEC_RESTORE = re.compile(r"^s_or_b64 exec, exec, ")
_EXECZ = re.compile(r"s_cbranch_execz (\.LBB\w+)")
_END = re.compile(r"^s_(cbranch|branch|endpgm|setpc)")


@dataclass
class Hit:
    kernel: str
    block: str
    line: int
    in_loop: bool
    spills: List[str] = field(default_factory=list)


def _is_spill(ins: str) -> bool:
    """A write of a vector register or of memory whose lanes follow exec: a
    spill store, or a copy into a vector or accumulation register.  Lane
    writes of scalar spills (v_writelane) ignore exec and do not count."""
    op = ins.split()[0]
    if op.startswith(("v_writelane", "v_readlane", "v_readfirstlane")):
        return False
    return op.startswith(("scratch_store", "buffer_store", "global_store", "flat_store",
                          "ds_write", "v_"))


def scan_text(text: str) -> List[Hit]:
    """Every spill placed in an execz join block ahead of its exec restore."""
    lines = text.split("\n")
    starts = [k for k, l in enumerate(lines) if _FUNC.match(l)] + [len(lines)]
    hits: List[Hit] = []
    for a, b in zip(starts, starts[1:]):
        kernel = _FUNC.match(lines[a]).group(1)
        body = lines[a:b]
        joins = set(_EXECZ.findall("\n".join(body)))
        block, in_loop, spills = None, False, []
        for k, raw in enumerate(body):
            m = _LABEL.match(raw)
            if m or _FALL.match(raw):
                block = m.group(1) if m else None
                in_loop = bool(m) and "Loop" in m.group(2)
                spills = []
                continue
            if block is None or block not in joins:
                continue
            ins = raw.strip()
            if not ins or ins.startswith(";"):
                continue
            if _EXEC_RESTORE.match(ins):
                if spills:
                    hits.append(Hit(kernel, block, a + k + 1, in_loop, spills))
                block = None
            elif _END.match(ins):
                block = None
            elif _is_spill(ins):
                spills.append(ins)
    return hits


def scan(path: str) -> List[Hit]:
    with open(path) as fh:
        return scan_text(fh.read())


def device_asm(outdir: str, jobs: int = 0) -> List[str]:
    """Device assembly of every translation unit of the library, in outdir."""
    inc = ["-I", os.path.join(build.ROOT, "include"), "-I", build.CSRC]
    outs = [os.path.join(outdir, os.path.basename(s)[:-4] + ".s") for s in build.SOURCES]
    cmds = [[build.HIPCC, *build.FLAGS, *inc, "--cuda-device-only", "-S", "-o", o, s]
            for s, o in zip(build.SOURCES, outs)]
    with ThreadPoolExecutor(max_workers=jobs or build._jobs()) as ex:
        procs = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
    for c, p in zip(cmds, procs):
        if p.returncode:
            sys.stderr.write(p.stderr)
            raise subprocess.CalledProcessError(p.returncode, c)
    return outs


def main() -> int:
    with tempfile.TemporaryDirectory() as d:
        hits = [h for p in device_asm(d) for h in scan(p)]
    for h in hits:
        where = "inside a loop" if h.in_loop else "outside loops"
        print(f"{h.kernel} {h.block} ({where}): {len(h.spills)} spill(s) ahead of the exec restore")
    return 1 if any(h.in_loop for h in hits) else 0


if __name__ == "__main__":
    sys.exit(main())
