"""Benchmark of the dense product C = A*B on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--paths fp64,split,...]

A step is one pass over every compute row of the hot path on resident,
seeded synthetic inputs:
  fp64     gemm_plain binary64, N = 2000, U[-1,1]                 (headline)
  split    gemm_split (split kernels + 3-term bfloat16 product), N = 2000
  split3   gemm_split3 (three-way split, 6-term bfloat16 product), N = 2000
  fp32     gemm_plain binary32, N = 2000
  bf16     gemm_plain bfloat16 inputs, binary32 output, N = 2000
  backward gemm_backward binary32 (dA and dB), N = 2048, dC = W
  grouped  512 products, N log-uniform in [10, 2000], binary64, one replay
           of the captured persistent launch (tuned policy); the same 512
           products as 512 single launches are timed after the step loop
           and reported beside it (loop_ms, speedup_vs_loop)
  grouped_fp32  the same batch in binary32
Each path is bracketed by HIP events on torch's current stream (the stream
the kernels run on); the step loop is bracketed by device synchronisation.
``value`` is the binary64 rate 2N^3/t at N = 2000; the split rate and every
other path are reported beside it with their normwise error against the
oracle's product of the same inputs. The oracle runs only in the CPU-baseline
leg: that leg times it (the paper's Algorithm 4 loop on all host threads) on
the N = 2000 binary64 product, keeps that product as the binary64 reference,
runs it once more on the binary32 inputs for the binary32, bfloat16 and split
paths, and serves every other stated error (full products up to 8.1e9
multiply-adds, 2000 sampled entries beyond). With --no-cpu-baseline the errors
fall back to host BLAS and ``rel_err_reference`` says so.
``roofline`` describes the binary64 kernel (MFMA bound).

Outside the timed step loop (each skippable):
  sweep     binary64 at the paper's sizes N = 10 ... 2000 plus 4096: median
            per-call rate (2N^3 and the paper's N^2(2N-1) count), error; for
            N <= 100 also single-call latency and 1000 back-to-back launches;
            and six rectangular binary64 shapes (m x k times k x n); the K
            split in binary32 and with bfloat16 inputs on two deep-K shapes
  transfer  N = 2000 binary64 with the operands on the host (pinned): H2D of
            A and B, the product, D2H of C, timed together (never ``value``)
  host      the host CPU (model, sockets, cores, threads), the single-thread
            oracle at N = 10 ... 2000, the Algorithm 4 loop on all host
            threads at N = 10 ... 2000 (4096 with --host-n4096) and on two
            threads at N = 2000 (the paper's two cores), with the GPU's
            binary64 speedup over each
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2516.6}   # TFLOP/s, dense MFMA
HBM_PEAK = 8000.0                                    # GB/s
METRIC = "GFLOP/s (2N^3/t) at N=2000 FP64 vs split-BF16, at stated rel. error"
ALL_PATHS = ["fp64", "split", "split3", "fp32", "bf16", "backward", "grouped", "grouped_fp32"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fp64_n2000.json")
# the binary64 kernel's code and the host choice of its tile shape
KERNEL_SOURCES = ["paper_1012_2273_amd/csrc/gemm_tile.hpp",
                  "paper_1012_2273_amd/csrc/gemm_tile_dma.hpp",
                  "paper_1012_2273_amd/csrc/kernels_plain.hip",
                  "paper_1012_2273_amd/csrc/gemm_api.hip"]


def kernel_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for_current_kernel():
    """HBM bytes per launch of the binary64 kernel from the committed counter
    summary, or None if absent or taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def host_threads():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _blas(A, B):
    """Host binary64 BLAS product of the exact inputs: the bench's error
    reference (the tests hold every path to the oracle itself)."""
    return np.matmul(np.asarray(A, np.float64), np.asarray(B, np.float64))


def _relerr(C, R):
    d = float(np.linalg.norm((np.asarray(C, np.float64) - R).ravel()))
    r = float(np.linalg.norm(R.ravel()))
    return d / r if r > 0 else d


def _entries(A, B, r, c):
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    return np.einsum("ij,ji->i", A[r, :], B[:, c])


class ErrRef:
    """Normwise relative error of a device result against a host product of
    the exact inputs. With the oracle (the CPU-baseline leg): its full product
    on all host threads up to FULL_LIMIT multiply-adds, its entries on a
    sample of 2000 positions beyond. Without it: host binary64 BLAS."""
    FULL_LIMIT = 8.1e9      # N = 2000 squares in full

    def __init__(self, oracle=None, threads=1):
        self.o, self.thr = oracle, threads
        if oracle is not None:
            self.kind = ("normwise, against the oracle's binary64 product of the same inputs "
                         f"(full product on {threads} host threads up to 8.1e9 multiply-adds, "
                         "2000 sampled entries beyond)")
        else:
            self.kind = ("normwise, against the host binary64 BLAS product of the same inputs "
                         "(the CPU-baseline leg, which holds the oracle, was skipped)")

    def product(self, A, B):
        return self.o.gemm_omp(A, B, self.thr) if self.o is not None else _blas(A, B)

    def err(self, C, A, B, full=None, seed=0):
        """C: device result on the host (the full matrix)."""
        if full is not None:
            return _relerr(C, full)
        m, k = A.shape
        n = B.shape[1]
        if self.o is None or float(m) * n * k <= self.FULL_LIMIT:
            return _relerr(C, self.product(A, B))
        g = np.random.Generator(np.random.PCG64(seed))
        r = g.integers(0, m, 2000)
        c = g.integers(0, n, 2000)
        return _relerr(np.asarray(C, np.float64)[r, c], self.o.gemm_entries(A, B, r, c))

    def entries(self, A, B, r, c):
        return self.o.gemm_entries(A, B, r, c) if self.o is not None else _entries(A, B, r, c)


def _median_ms(pairs):
    return float(np.median([a.elapsed_time(b) for a, b in pairs]))


def fp64_sweep(G, torch, dev, stream, inputs, ref, full=None):
    """The paper's size sweep (Tables 1-2: N = 100 ... 2000) plus N = 10 and
    4096, binary64, inputs resident."""
    out = {}
    for n in (10, 100, 500, 1000, 2000, 4096):
        print(f"sweep: binary64 N={n}", file=sys.stderr, flush=True)
        A, B = inputs.uniform_square(n, inputs.seed_for(1, n))
        Ad, Bd = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
        Cd = torch.empty((n, n), dtype=torch.float64, device=dev)
        # warm up for at least 30 ms of back-to-back calls: after the thousands
        # of tiny launches of the small sizes the clock needs time to come back
        t_end = time.perf_counter() + 0.03
        while True:
            for _ in range(5):
                G.gemm_plain(Ad, Bd, Cd)
            torch.cuda.synchronize()
            if time.perf_counter() >= t_end:
                break
        reps = 20 if n >= 1000 else 200
        pairs = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            G.gemm_plain(Ad, Bd, Cd)
            e1.record(stream)
            pairs.append((e0, e1))
        torch.cuda.synchronize()
        t = _median_ms(pairs) * 1e-3
        d = {"ms": round(t * 1e3, 5), "gflops": round(2.0 * n ** 3 / t / 1e9, 2),
             "gflops_paper_count": round(n * n * (2 * n - 1) / t / 1e9, 2),
             "frac_peak": round(2.0 * n ** 3 / t / 1e12 / PEAK["f64"], 4)}
        if n <= 100:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(1000):
                G.gemm_plain(Ad, Bd, Cd)
            e1.record(stream)
            torch.cuda.synchronize()
            per = e0.elapsed_time(e1) * 1e-3 / 1000
            d["latency_us"] = round(t * 1e6, 2)
            d["amortised_us"] = round(per * 1e6, 3)
            d["amortised_gflops"] = round(2.0 * n ** 3 / per / 1e9, 3)
            d["amortised_gbs"] = round(24.0 * n * n / per / 1e9, 2)   # A, B, C once
        if ref is not None:
            C = Cd.cpu().numpy()
            d["rel_err"] = float(f"{ref.err(C, A, B, full=(full or {}).get(n)):.3e}")
        out[str(n)] = d
        del Ad, Bd, Cd
    return out


RECT_SHAPES = [(2000, 1000, 3000), (3000, 3000, 3000), (8192, 512, 8192), (512, 8192, 8192),
               (4096, 4096, 512), (256, 256, 65536)]


def _median_call_ms(fn, torch, stream):
    """Median per-call time of fn() after >= 30 ms of warm-up, HIP events
    on the stream the kernels run on."""
    t_end = time.perf_counter() + 0.03
    while True:
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        if time.perf_counter() >= t_end:
            break
    pairs = []
    for _ in range(10):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        pairs.append((e0, e1))
    torch.cuda.synchronize()
    return _median_ms(pairs)


def rect_sweep(G, torch, dev, stream, inputs, ref):
    """Rectangular binary64 products (m x k times k x n, the paper's problem
    statement), median per-call rate after >= 30 ms of warm-up; where
    gemm_plain_ksplit splits the K loop (too few output tiles for the
    device), its rate beside it ("ksplit")."""
    out = {}
    for m, n, k in RECT_SHAPES:
        print(f"sweep: binary64 {m}x{n}x{k}", file=sys.stderr, flush=True)
        A, B = inputs.uniform_mnk(m, n, k, 5_000_000 + m + n + k)
        Ad, Bd = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
        Cd = torch.empty((m, n), dtype=torch.float64, device=dev)
        t = _median_call_ms(lambda: G.gemm_plain(Ad, Bd, Cd), torch, stream) * 1e-3
        d = {"ms": round(t * 1e3, 5), "gflops": round(2.0 * m * n * k / t / 1e9, 2),
             "frac_peak": round(2.0 * m * n * k / t / 1e12 / PEAK["f64"], 4)}
        full = None
        if ref is not None:
            if ref.o is None or float(m) * n * k <= ref.FULL_LIMIT:
                full = ref.product(A, B)
            d["rel_err"] = float(f"{ref.err(Cd.cpu().numpy(), A, B, full=full, seed=m + n):.3e}")
        need = G.gemm_plain_ksplit_workspace_size(G.GEMM_F64, m, n, k)
        if need > 0:
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
            tk = _median_call_ms(lambda: G.gemm_plain_ksplit(Ad, Bd, Cd, ws), torch, stream) * 1e-3
            ks = {"ms": round(tk * 1e3, 5), "gflops": round(2.0 * m * n * k / tk / 1e9, 2),
                  "frac_peak": round(2.0 * m * n * k / tk / 1e12 / PEAK["f64"], 4),
                  "workspace_bytes": need}
            if ref is not None:
                ks["rel_err"] = float(f"{ref.err(Cd.cpu().numpy(), A, B, full=full, seed=m + n):.3e}")
            d["ksplit"] = ks
            del ws
        out[f"{m}x{n}x{k}"] = d
        del Ad, Bd, Cd
    return out


KSPLIT_32_16 = [(1024, 1024, 8192), (256, 256, 65536)]


def ksplit_sweep(G, torch, dev, stream, inputs, ref):
    """gemm_plain against gemm_plain_ksplit in binary32 and with bfloat16
    inputs on deep-K shapes; bf16 errors against the oracle of the rounded
    inputs (``rel_err``) and of the binary32 data (``rel_err_path``)."""
    out = {}
    for m, n, k in KSPLIT_32_16:
        print(f"sweep: K split {m}x{n}x{k} binary32 and bf16", file=sys.stderr, flush=True)
        A, B = inputs.uniform_mnk(m, n, k, 6_000_000 + m + n + k, dtype=np.float32)
        A32d, B32d = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
        for name, Ad, Bd in (("f32", A32d, B32d),
                             ("bf16", A32d.to(torch.bfloat16), B32d.to(torch.bfloat16))):
            Cd = torch.empty((m, n), dtype=torch.float32, device=dev)
            fl = 2.0 * m * n * k
            tp = _median_call_ms(lambda: G.gemm_plain(Ad, Bd, Cd), torch, stream) * 1e-3
            need = G.gemm_plain_ksplit_workspace_size(
                G.GEMM_F32 if name == "f32" else G.GEMM_BF16, m, n, k)
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
            tk = _median_call_ms(lambda: G.gemm_plain_ksplit(Ad, Bd, Cd, ws), torch, stream) * 1e-3
            d = {"plain_gflops": round(fl / tp / 1e9, 2), "ksplit_ms": round(tk * 1e3, 5),
                 "ksplit_gflops": round(fl / tk / 1e9, 2), "workspace_bytes": need}
            if ref is not None:
                C = Cd.cpu().double().numpy()
                if name == "bf16":
                    Ar, Br = Ad.double().cpu().numpy(), Bd.double().cpu().numpy()
                    d["rel_err"] = float(f"{ref.err(C, Ar, Br, seed=m + k):.3e}")
                    d["rel_err_path"] = float(f"{ref.err(C, A, B, seed=m + k):.3e}")
                else:
                    d["rel_err"] = float(f"{ref.err(C, A, B, seed=m + k):.3e}")
            out[f"{name}_{m}x{n}x{k}"] = d
            del ws, Cd
    return out


PRECISION_SIZES = (4096, 8192)


def precision_sweep(G, torch, dev, stream, inputs, ref):
    """The precision study's larger sizes: binary32 inputs (U[-1, 1]) as plain
    binary32, plain bf16 (errors against the oracle of the rounded inputs,
    ``rel_err``, and of the binary32 data, ``rel_err_path``), the two-way and
    the three-way split (against the oracle of the binary32 data); nominal
    2N^3/t, each path's median over back-to-back calls."""
    out = {}
    for n in PRECISION_SIZES:
        print(f"sweep: precision paths N={n}", file=sys.stderr, flush=True)
        A, B = inputs.uniform_square(n, inputs.seed_for(2, n), dtype=np.float32)
        Ad, Bd = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
        Ab, Bb = Ad.to(torch.bfloat16), Bd.to(torch.bfloat16)
        Cd = torch.empty((n, n), dtype=torch.float32, device=dev)
        ws2 = torch.empty(G.gemm_split_workspace_size(n, n, n), dtype=torch.uint8, device=dev)
        ws3 = torch.empty(G.gemm_split3_workspace_size(n, n, n), dtype=torch.uint8, device=dev)
        fl = 2.0 * n ** 3
        row = {}
        for name, fn in (("fp32", lambda: G.gemm_plain(Ad, Bd, Cd)),
                         ("bf16", lambda: G.gemm_plain(Ab, Bb, Cd)),
                         ("split", lambda: G.gemm_split(Ad, Bd, Cd, ws2)),
                         ("split3", lambda: G.gemm_split3(Ad, Bd, Cd, ws3))):
            t = _median_call_ms(fn, torch, stream) * 1e-3
            d = {"ms": round(t * 1e3, 4), "gflops": round(fl / t / 1e9, 2)}
            if ref is not None:
                fn()
                torch.cuda.synchronize()
                C = Cd.cpu().double().numpy()
                if name == "bf16":
                    Ar, Br = Ab.double().cpu().numpy(), Bb.double().cpu().numpy()
                    d["rel_err"] = float(f"{ref.err(C, Ar, Br, seed=n + 1):.3e}")
                    d["rel_err_path"] = float(f"{ref.err(C, A, B, seed=n + 1):.3e}")
                else:
                    d["rel_err"] = float(f"{ref.err(C, A, B, seed=n + 1):.3e}")
            row[name] = d
        out[str(n)] = row
        del Ad, Bd, Ab, Bb, Cd, ws2, ws3
    return out


def transfer_inclusive(G, torch, dev, stream, A, B, C_resident, reps=10):
    """N = 2000 binary64 with the operands starting and ending in pinned host
    memory: H2D of A and B, the product, D2H of C on one stream."""
    n = A.shape[0]
    Ah = torch.empty((n, n), dtype=torch.float64, pin_memory=True)
    Bh = torch.empty((n, n), dtype=torch.float64, pin_memory=True)
    Ch = torch.empty((n, n), dtype=torch.float64, pin_memory=True)
    Ah.copy_(torch.from_numpy(A))
    Bh.copy_(torch.from_numpy(B))
    Ad = torch.empty((n, n), dtype=torch.float64, device=dev)
    Bd = torch.empty_like(Ad)
    Cd = torch.empty_like(Ad)
    rows = []
    for i in range(reps + 2):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        Ad.copy_(Ah, non_blocking=True)
        Bd.copy_(Bh, non_blocking=True)
        ev[1].record(stream)
        G.gemm_plain(Ad, Bd, Cd)
        ev[2].record(stream)
        Ch.copy_(Cd, non_blocking=True)
        ev[3].record(stream)
        if i >= 2:
            rows.append(ev)
    torch.cuda.synchronize()
    h2d = float(np.median([e[0].elapsed_time(e[1]) for e in rows]))
    mm = float(np.median([e[1].elapsed_time(e[2]) for e in rows]))
    d2h = float(np.median([e[2].elapsed_time(e[3]) for e in rows]))
    tot = float(np.median([e[0].elapsed_time(e[3]) for e in rows]))
    return {"N": n, "ms_total": round(tot, 4), "ms_h2d": round(h2d, 4), "ms_product": round(mm, 4),
            "ms_d2h": round(d2h, 4), "gflops": round(2.0 * n ** 3 / (tot * 1e-3) / 1e9, 2),
            "h2d_gbs": round(16.0 * n * n / (h2d * 1e-3) / 1e9, 2),
            "d2h_gbs": round(8.0 * n * n / (d2h * 1e-3) / 1e9, 2),
            "matches_resident": bool(torch.equal(Ch, C_resident.cpu()))}


def lscpu():
    """Host CPU model, sockets, cores per socket, threads per core and CPU
    count from lscpu (else /proc/cpuinfo), and the threads this process may use."""
    info = {}
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        keys = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket":
                "cores_per_socket", "Thread(s) per core": "threads_per_core", "CPU(s)": "cpus"}
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in keys and keys[k.strip()] not in info:
                v = v.strip()
                info[keys[k.strip()]] = int(v) if v.isdigit() else v
    except (OSError, ValueError):
        pass
    if "model" not in info:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        info["model"] = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    info["threads_available"] = host_threads()
    return info


def _host_time(fn, min_s=0.05):
    """Median wall time of fn() over repeats totalling at least min_s."""
    runs = []
    t_end = time.perf_counter() + min_s
    while not runs or (time.perf_counter() < t_end and len(runs) < 1000):
        t0 = time.perf_counter()
        fn()
        runs.append(time.perf_counter() - t0)
    return float(np.median(runs))


def host_info(oracle, inputs, gpu_sweep=None, alg4_sizes=(10, 100, 500, 1000, 2000)):
    """The host CPU and the paper's CPU programs on it: the oracle on one
    thread at the paper's sizes N = 10 ... 2000, the paper's Algorithm 4 (rows
    split statically over threads) on all host threads at N = 10 ... 2000 (and
    4096 with --host-n4096: the loop walks B by columns, which at N = 4096 no
    longer fits the host caches and takes minutes) and on two threads at
    N = 2000 (the paper's two cores). Inputs are made before the
    clock starts, as the paper times only the product. Rates at 2N^3 and at the
    paper's N^2(2N-1) count; ``gpu_speedup`` is the host time over the GPU's
    binary64 time at the same N (the sweep's median per call)."""
    thr = host_threads()

    t_host0 = time.perf_counter()

    def row(n, threads):
        print(f"host: N={n} on {threads} thread(s) "
              f"({time.perf_counter() - t_host0:.1f} s into the host sweep)", file=sys.stderr,
              flush=True)
        A, B = inputs.uniform_square(n, inputs.seed_for(1, n))
        if threads == 1:
            t = _host_time(lambda: oracle.gemm(A, B))
        else:
            t = _host_time(lambda: oracle.gemm_omp(A, B, threads))
        d = {"s": float(f"{t:.4g}"), "gflops": round(2.0 * n ** 3 / t / 1e9, 3),
             "gflops_paper_count": round(n * n * (2 * n - 1) / t / 1e9, 3)}
        g = (gpu_sweep or {}).get(str(n))
        if g:
            d["gpu_speedup"] = round(t / (g["ms"] * 1e-3), 1)
        return d

    return {"cpu": lscpu(),
            "oracle_1thread": {str(n): row(n, 1) for n in (10, 100, 500, 1000, 2000)},
            f"alg4_{thr}threads": {str(n): row(n, thr) for n in alg4_sizes},
            "alg4_2threads": {"2000": row(2000, 2)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--paths", default=",".join(ALL_PATHS))
    ap.add_argument("--n", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the error check")
    ap.add_argument("--tile-config", type=int, default=-1,
                    help="force one tile configuration id for single-product launches")
    ap.add_argument("--no-sweep", action="store_true", help="skip the binary64 size sweep")
    ap.add_argument("--no-transfer", action="store_true", help="skip the host-buffer timing")
    ap.add_argument("--host-n4096", action="store_true",
                    help="also time the paper's Algorithm 4 on all host threads at N = 4096 "
                         "(several minutes of host work)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a device-to-device copy of 512 MiB (3 times) so that "
                         "counter runs can scale FETCH_SIZE/WRITE_SIZE to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has "
              "no multi-GPU path: the product would shard by row blocks of A and C "
              "(see the design notes), which is not built here.", file=sys.stderr)
        sys.exit(2)
    paths = [p for p in args.paths.split(",") if p]
    for p in paths:
        if p not in ALL_PATHS:
            sys.exit(f"unknown path {p}")

    import torch

    import paper_1012_2273_amd as G
    from paper_1012_2273_amd import inputs

    if not os.path.exists(G._lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    G.load()
    if args.tile_config >= 0:
        G.force_tile_config(args.tile_config)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    N = args.n
    log = lambda *a: print(*a, file=sys.stderr, flush=True)

    # ---------------------------------------------------------------- inputs
    host = {}
    work = {}          # path -> (callable, algorithmic flops per call)
    A64, B64 = inputs.uniform_square(N, inputs.seed_for(1, N))
    host["fp64"] = (A64, B64)
    A64d, B64d = torch.from_numpy(A64).to(dev), torch.from_numpy(B64).to(dev)
    C64d = torch.empty((N, N), dtype=torch.float64, device=dev)
    work["fp64"] = (lambda: G.gemm_plain(A64d, B64d, C64d), 2.0 * N ** 3)

    if any(p in paths for p in ("split", "split3", "fp32", "bf16")):
        A32, B32 = inputs.uniform_square(N, inputs.seed_for(2, N), dtype=np.float32)
        host["f32"] = (A32, B32)
        A32d, B32d = torch.from_numpy(A32).to(dev), torch.from_numpy(B32).to(dev)
        Csd = torch.empty((N, N), dtype=torch.float32, device=dev)
        ws = torch.empty(G.gemm_split_workspace_size(N, N, N), dtype=torch.uint8, device=dev)
        work["split"] = (lambda: G.gemm_split(A32d, B32d, Csd, ws), 2.0 * N ** 3)
        C3d = torch.empty((N, N), dtype=torch.float32, device=dev)
        ws3 = torch.empty(G.gemm_split3_workspace_size(N, N, N), dtype=torch.uint8, device=dev)
        work["split3"] = (lambda: G.gemm_split3(A32d, B32d, C3d, ws3), 2.0 * N ** 3)
        C32d = torch.empty((N, N), dtype=torch.float32, device=dev)
        work["fp32"] = (lambda: G.gemm_plain(A32d, B32d, C32d), 2.0 * N ** 3)
        A16d, B16d = A32d.to(torch.bfloat16), B32d.to(torch.bfloat16)
        C16d = torch.empty((N, N), dtype=torch.float32, device=dev)
        work["bf16"] = (lambda: G.gemm_plain(A16d, B16d, C16d), 2.0 * N ** 3)

    if "backward" in paths:
        NB = 2048
        Ab, Bb, Wb = inputs.uniform((NB, NB), inputs.seed_for(4, NB), np.float32, 3)
        host["backward"] = (Ab, Bb, Wb)
        Abd, Bbd, Wbd = (torch.from_numpy(x).to(dev) for x in (Ab, Bb, Wb))
        bw_out = {}

        def run_bw():
            bw_out["d"] = G.gemm_backward(Abd, Bbd, Wbd)
        work["backward"] = (run_bw, 2 * 2.0 * NB ** 3)

    gp = {}   # grouped path -> its plan, device operands and host problems
    for gpath, gdt in (("grouped", np.float64), ("grouped_fp32", np.float32)):
        if gpath not in paths:
            continue
        log(f"generating 512-problem batch ({gpath})")
        sizes = inputs.batch_sizes(512, 3_000_000)
        gA, gB, gprobs = [], [], []
        for i, n in enumerate(sizes):
            A, B = inputs.batch_problem(i, int(n), 3_000_000, gdt)
            gprobs.append((A, B))
            gA.append(torch.from_numpy(A).to(dev))
            gB.append(torch.from_numpy(B).to(dev))
        import tempfile
        cache = os.path.join(tempfile.mkdtemp(prefix="gemm_tune_"), "tune_cache.json")
        t0 = time.time()
        plan = G.GroupedPlan(gA, gB, autotune=True, tune_cache=cache)
        log(f"{gpath} plan (autotune) {time.time() - t0:.2f}s; tiles/policy {plan.info()}")
        gp[gpath] = {"plan": plan, "A": gA, "B": gB, "sizes": sizes, "probs": gprobs}
        work[gpath] = (plan.run, float(sum(2 * int(n) ** 3 for n in sizes)))

    order = [p for p in ALL_PATHS if p in paths]

    if args.copy_calibration:
        # a plain copy kernel of known size: reads and writes 512 MiB each
        src = torch.empty(512 << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 512 MiB device-to-device copies")
        del src, dst

    # ---------------------------------------------------------------- timing
    stream = torch.cuda.current_stream(dev)
    log(f"timing: {args.warmup} warm-up and {args.steps} timed steps of {order}")
    for _ in range(args.warmup):
        for p in order:
            work[p][0]()
    torch.cuda.synchronize()
    evs = {p: [] for p in order}
    t_wall0 = time.perf_counter()
    for _ in range(args.steps):
        for p in order:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            work[p][0]()
            e1.record(stream)
            evs[p].append((e0, e1))
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall0
    ms = {p: float(np.mean([a.elapsed_time(b) for a, b in evs[p]])) for p in order}
    ms_min = {p: float(np.min([a.elapsed_time(b) for a, b in evs[p]])) for p in order}

    # ------------------------------------- grouped versus one launch per product
    loop = {}
    for gpath, g in gp.items():
        gC = [torch.empty_like(a) for a in g["A"]]

        def run_loop():
            for a, b, c in zip(g["A"], g["B"], gC):
                G.gemm_plain(a, b, c)
        run_loop()
        torch.cuda.synchronize()
        le = []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run_loop()
            e1.record(stream)
            le.append((e0, e1))
        torch.cuda.synchronize()
        loop[gpath] = float(np.mean([a.elapsed_time(b) for a, b in le]))
        del gC

    # ---------------------------------------------------------- cpu baseline
    # The CPU-baseline leg: the oracle timed on the host cores, and the
    # reference products every stated error is taken against.
    cpu = None
    ref = None
    ref64 = None
    if not args.no_cpu_baseline:
        import oracle
        thr = host_threads()
        log(f"cpu baseline: oracle N={N} on {thr} threads, about 10 s")
        ref = ErrRef(oracle, thr)
        A, B = host["fp64"]
        runs = []
        t_start = time.perf_counter()
        # repeat the full product for about 10 s of host work (at least 3 runs)
        while len(runs) < 3 or (time.perf_counter() - t_start < 10.0 and len(runs) < 200):
            t0 = time.perf_counter()
            ref64 = oracle.gemm_omp(A, B, thr)
            runs.append(time.perf_counter() - t0)
        tc = float(np.median(runs))
        cpu = {"value": round(2.0 * N ** 3 / tc / 1e9, 3), "unit": "GFLOP/s", "cores": thr,
               "kind": "oracle",
               "sample": f"the full N={N} binary64 product, oracle loop (row, column, "
                         f"reduction; no FMA) with rows split statically over {thr} threads "
                         f"as in the paper's Algorithm 4; median of {len(runs)} runs "
                         f"({sum(runs):.1f} s of host work), {tc:.2f} s each"}
    elif not args.no_check:
        ref = ErrRef(None)
    if args.no_check:
        ref = None

    # ---------------------------------------------------------- error check
    errs = {}
    if ref is not None:
        log("errors against the reference products")
        A, B = host["fp64"]
        errs["fp64"] = ref.err(C64d.cpu().numpy(), A, B, full=ref64)
        if "f32" in host:
            A, B = host["f32"]
            ref32 = ref.product(A, B)       # one oracle run on the binary32 inputs
            if "split" in order:
                errs["split"] = _relerr(Csd.cpu().double().numpy(), ref32)
            if "split3" in order:
                errs["split3"] = _relerr(C3d.cpu().double().numpy(), ref32)
            if "fp32" in order:
                errs["fp32"] = _relerr(C32d.cpu().double().numpy(), ref32)
            if "bf16" in order:
                errs["bf16"] = _relerr(C16d.cpu().double().numpy(), ref32)
            del ref32
        if "backward" in order:
            Ab, Bb, Wb = host["backward"]
            g = np.random.Generator(np.random.PCG64(1))
            r = g.integers(0, Ab.shape[0], 400)
            c = g.integers(0, Ab.shape[0], 400)
            dA, dB = (t.cpu().double().numpy() for t in bw_out["d"])
            eA = _relerr(dA[r, c], ref.entries(Wb, np.ascontiguousarray(Bb.T), r, c))
            eB = _relerr(dB[r, c], ref.entries(np.ascontiguousarray(Ab.T), Wb, r, c))
            errs["backward"] = max(eA, eB)
        for gpath, gd in gp.items():
            worst = 0.0
            g = np.random.Generator(np.random.PCG64(2))
            for i in range(0, len(gd["sizes"]), 4):
                A, B = gd["probs"][i]
                n = int(gd["sizes"][i])
                r = g.integers(0, n, 40)
                c = g.integers(0, n, 40)
                got = gd["plan"].Cs[i].cpu().double().numpy()[r, c]
                worst = max(worst, _relerr(got, ref.entries(A, B, r, c)))
            errs[gpath] = worst

    # ------------------------------------------- outside the timed step loop
    sweep = rect = ksw = prec = None
    if not args.no_sweep:
        sweep = fp64_sweep(G, torch, dev, stream, inputs, ref, full={N: ref64})
        rect = rect_sweep(G, torch, dev, stream, inputs, ref)
        ksw = ksplit_sweep(G, torch, dev, stream, inputs, ref)
        prec = precision_sweep(G, torch, dev, stream, inputs, ref)
    xfer = None
    if not args.no_transfer:
        A, B = host["fp64"]
        xfer = transfer_inclusive(G, torch, dev, stream, A, B, C64d)
    hinfo = None
    if not args.no_cpu_baseline:
        import oracle     # the CPU-baseline leg: the oracle timed on the host
        hinfo = host_info(oracle, inputs, sweep,
                          (10, 100, 500, 1000, 2000) + ((4096,) if args.host_n4096 else ()))

    # ---------------------------------------------------------- report
    paths_out = {}
    for p in order:
        flops = work[p][1]
        d = {"ms": round(ms[p], 5), "ms_min": round(ms_min[p], 5),
             "gflops": round(flops / (ms[p] * 1e-3) / 1e9, 2)}
        if p in errs:
            d["rel_err"] = float(f"{errs[p]:.3e}")
        paths_out[p] = d
    for gpath, lm in loop.items():
        paths_out[gpath]["loop_ms"] = round(lm, 4)
        paths_out[gpath]["loop_gflops"] = round(work[gpath][1] / (lm * 1e-3) / 1e9, 2)
        paths_out[gpath]["speedup_vs_loop"] = round(lm / ms[gpath], 3)
    if "split" in paths_out:
        paths_out["split"]["mfma_util_bf16"] = round(
            6.0 * N ** 3 / (ms["split"] * 1e-3) / 1e12 / PEAK["bf16"], 4)
    # a run restricted to other paths (--paths) reports no headline value
    t_fp64 = ms["fp64"] * 1e-3 if "fp64" in ms else float("nan")
    achieved = 2.0 * N ** 3 / t_fp64 / 1e12
    traffic = traffic_for_current_kernel()
    line = {
        "metric": METRIC,
        "value": round(2.0 * N ** 3 / t_fp64 / 1e9, 2) if "fp64" in ms else None,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded U[-1,1], row-major)",
        "config": {"workload": f"square dense product N={N}: binary64 (value) and binary32 "
                               "3-term bfloat16 split, plus the other paths of the step",
                   "N": N, "paths": order},
        "split_bf16": {"value": paths_out.get("split", {}).get("gflops"),
                       "rel_err": paths_out.get("split", {}).get("rel_err"),
                       "vs_fp64": (round(ms["fp64"] / ms["split"], 2)
                                 if "split" in ms and "fp64" in ms else None)},
        "fp64_rel_err": paths_out.get("fp64", {}).get("rel_err"),
        "rel_err_reference": ref.kind if ref is not None else None,
        "paths": paths_out,
        "roofline": ({"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["f64"],
                      "unit": "TFLOP/s", "frac": round(achieved / PEAK["f64"], 4),
                      "traffic": traffic} if "fp64" in ms else None),
        "cpu_baseline": cpu,
        "sweep_fp64": sweep,
        "sweep_rect_fp64": rect,
        "sweep_ksplit_f32_bf16": ksw,
        "sweep_precision": prec,
        "transfer_inclusive": xfer,
        "host": hinfo,
    }
    print(json.dumps(line), flush=True)
    for g in gp.values():
        g["plan"].close()


if __name__ == "__main__":
    main()
