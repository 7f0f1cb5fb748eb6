"""Build libparafac2.so (HIP kernels + host runtime + C ABI) for gfx950 in-tree.

The library is plain HIP C++ with an extern "C" interface; it does not link
against torch.  Run `python -m paper_1703_04219_amd.build` or call build().
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libparafac2.so")
SOURCES = ["p2_kernels.hip", "p2_capi.hip", "p2_server.hip", "p2_baseline.hip"]
# The rank-templated kernels: p2_ranks.hip is compiled once per subset of the
# ranks (P2_SHARD_RANKS), so that the subsets compile in parallel.  The ranks
# must be those of P2_RANKS in p2_rank_impl.h; a mismatch fails the link.
RANK_SOURCE = "p2_ranks.hip"
RANKS = tuple(range(1, 41))
N_SHARDS = 8

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PARAFAC2_ARCH", "gfx950")

CFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-munsafe-fp-atomics",
    # packed FP32 VALU ops are not emitted (they are unreliable on this part)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _rank_cost(r: int) -> float:
    """Rough hipcc seconds for one rank's kernels: the unrolled R x R loops
    grow with R, and ranks 17-20 also build warm-started Procrustes kernels
    at two lane groups per rank."""
    return 3.0 + 0.4 * r + (2.0 if 16 < r <= 20 else 0.0)


def rank_shards(n: int = N_SHARDS) -> list[list[int]]:
    """Split RANKS into n subsets of about equal compile time (largest first,
    each to the subset with the least so far)."""
    shards: list[list[int]] = [[] for _ in range(n)]
    load = [0.0] * n
    for r in sorted(RANKS, key=_rank_cost, reverse=True):
        i = min(range(n), key=load.__getitem__)
        shards[i].append(r)
        load[i] += _rank_cost(r)
    return [sorted(sh) for sh in shards if sh]


def _jobs() -> list[tuple[str, str, list[str]]]:
    jobs = [(src, os.path.splitext(src)[0] + ".o", []) for src in SOURCES]
    for i, sh in enumerate(rank_shards()):
        ranks = " ".join(f"X({r})" for r in sh)
        jobs.append((RANK_SOURCE, f"p2_ranks_{i}.o", [f"-DP2_SHARD_RANKS(X)={ranks}"]))
    return jobs


def _compile(job: tuple[str, str, list[str]]) -> str:
    src, name, extra = job
    obj = os.path.join(BUILD, name)
    cmd = [HIPCC, *CFLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} {' '.join(extra)}:\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = _jobs()
    with cf.ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, jobs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
