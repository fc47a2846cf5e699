"""Benchmark of the MI355X hash-map hot path.

One step = one pass of the plain-map workload at scale on one GPU:
  clear -> insert 10M int32x3 keys with f32 x C values (distinct ratio rho)
        -> find 10M keys (50% hits, indices and masks)
        -> erase 5M keys
with every input already resident in HBM.  `value` is key operations per
second over the whole step (insert + find + erase positions / step time).

Per-kernel durations come from HIP events the library records around each
launch on the launch stream (ash_profile_enable) during the timed steps.  The
roofline covers the dominant operation, insert (claim + commit): bytes per
position under the granule accounting (every unavoidable random access one
DRAM granule, g = 128 B measured on MI355X by `--workload access`) times the
positions of one call, over the summed average durations of its kernels.
`accounting` gives insert, find and erase under the payload and granule
accountings (g = 128 and g = 64).  `traffic` is the L2-to-fabric bytes per
insert measured with rocprofv3 counters on the same sources and workload
(null otherwise).  `served` runs the served map beside the plain path on
the served request stream: the plain path's mixed throughput (each request
a direct call, back to back on one stream), the server's burst capacity,
and offered loads of 0.5x and 0.9x of that plain-path throughput.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--rho 0.5] [--channels 8]
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

# Cost of one random access on MI355X, measured by `--workload access` (the
# access-cost summary in profiles/): every random read of 4 to 128 bytes is
# one 128-byte request from L2 to memory (TCC_EA0_RDREQ_128B), and on a
# 16 GiB table random reads of 16 B and of 128 B run at the same 49 G/s
# (256 B reads at half that), so the DRAM granule of a random access is
# 128 bytes.  A device-scope 64-bit CAS is one 64-byte atomic request at the
# memory side, a 32-bit atomic one 32-byte request, and a random 16-byte
# store one 32-byte write request.
GRANULE_B = 128
READ_LINE = GRANULE_B
CAS64 = 64
ATOM32 = 32
STORE = 32


def op_bytes(op, g, u=0.0, eta=0.0, e=0.0, C=8):
    """Bytes per operation of a random-access hash map keyed by 12-byte keys
    with 4-byte indices, 1-byte masks and 8-byte slot pairs (tag word, state),
    under two accountings: payload (the bytes the method touches) and granule
    (each unavoidable random access counted as one DRAM granule g).
    u = fraction of insert positions that hold a new key, eta = find hit
    rate, e = fraction of erase positions that free an index, C = float32
    value channels.

    insert  payload 25 + 12(1-u) + u(24 + 8C): key 12 in, index 4 and mask 1
            out, the slot pair 8; a key already present is compared (12); a
            new key writes its slot pair 8, k^B 12, reads its heap entry 4
            and moves its value row 4C in and 4C out.
            granule 17 + 2g + u(16 + 8C): streams 17, the probe window and a
            second random access (the claim of a new key, the key compare of
            an old one), k^B 12 + heap 4 + the value row per new key.
    find    payload 25 + 12 eta; granule 17 + g(1 + eta) (a separate k^B read
            per hit); find_in_slot: 17 + g for a table that holds the key in
            its slot (this one), where a hit needs no second access.
    erase   payload 37 + 13e; granule 13 + 3g + 5e."""
    if op == "insert":
        return {"payload": 25 + 12 * (1 - u) + u * (24 + 8 * C), "granule": 17 + 2 * g + u * (16 + 8 * C)}
    if op == "find":
        return {"payload": 25 + 12 * eta, "granule": 17 + g * (1 + eta)}
    if op == "find_in_slot":
        return {"payload": 25 + 12 * eta, "granule": 17 + g}
    if op == "erase":
        return {"payload": 37 + 13 * e, "granule": 13 + 3 * g + 5 * e}
    raise ValueError(op)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None

# HBM bytes per launch at the default workload, per table shape (probe_group,
# bucket_width, max_load), from rocprofv3 FETCH_SIZE and WRITE_SIZE runs
# scaled by what they read for the library's streaming copy of 128 MiB
# (fetch x1.9996, write x1.0000).  They hold for the kernel sources with these
# SHA-256 digests only: traffic is reported as null for any other sources,
# workload or shape.
MEASURED_TRAFFIC = {
    (1, 2, 0.85): {"claim": 2.5077e9, "commit": 0.9239e9, "find": 1.5109e9, "erase_mark": 0.9202e9,
                   "erase_commit": 0.1806e9},
    (1, 4, 0.85): {"claim": 2.4555e9, "commit": 0.9234e9, "find": 1.4713e9, "erase_mark": 0.8993e9,
                   "erase_commit": 0.1803e9},
    (1, 2, 0.7): {"claim": 2.4859e9, "commit": 0.9231e9, "find": 1.4886e9, "erase_mark": 0.9216e9,
                  "erase_commit": 0.1802e9},
    (4, 4, 0.5): {"claim": 2.4237e9, "commit": 0.9234e9, "find": 1.4429e9, "erase_mark": 0.8949e9,
                  "erase_commit": 0.1804e9},
}
# The same for the neighbor search (radius 1 over the 4.8M surface cells,
# one lane per key, W = 4, max load 0.5, queries in first-appearance order),
# on the same kernel sources.
MEASURED_TRAFFIC_NEIGHBORS = 18.53e9
MEASURED_SOURCES = {
    "ash_kernels.hip": "c7732ebd7ee6e5352dfa1a20592b895ae015cf756efa188568efbcf3980a2bb3",
    "ash_device.hpp": "cf221c03b17cac844c99a3452aaa61c4993f086eb01d64fc70f059fedac8000e",
}


def sources_measured():
    """True when the kernel sources are the ones the counters were taken on."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2110_00511_amd", "csrc")
    for name, digest in MEASURED_SOURCES.items():
        with open(os.path.join(csrc, name), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return False
    return True


def measured_traffic(args, shape):
    """The counters' bytes per kernel when the kernels, the workload and the
    table shape are ones they were taken on, else None."""
    if not sources_measured() or (args.rho, args.channels) != (0.5, 8) or args.lds_dedup or args.sorted_keys:
        return None
    for (pg, bw, ml), per_kernel in MEASURED_TRAFFIC.items():
        if (pg, bw) == tuple(shape[:2]) and abs(ml - shape[2]) < 1e-4:
            return per_kernel
    return None


def kernel_bytes(name, n, u, d, e, channels, inline_values=True):
    """Algorithmic DRAM bytes of one launch over n positions.

    u = fraction of positions holding a new key, d = fraction that are later
    duplicates of a new key in the same batch, e = fraction of erase positions
    that free an index, C = float channels per value row.

    claim        : key 12 (stream) + slot window (line) + claim CAS for new keys
                   + one read of the first occurrence's key per in-batch duplicate
    commit       : idx 4 + mask 1 (stream) + per new key: k^B 12, heap 4, and
                   either value read 4C and write 4C (rows copied inside the
                   commit) or the winner list 4 (rows copied by `values`)
    values       : per new key: winner list 4, heap 4, value read 4C and write 4C
    find         : key 12 + idx 4 + mask 1 (stream) + slot window (line)
    erase_mark   : key 12 (stream) + slot window (line) + owner election (64-bit atomic)
    erase_commit : mask 1 (stream) + per freed index: heap 4 + tombstone store
    """
    if name == "claim":
        return n * (12 + READ_LINE + u * CAS64 + d * READ_LINE)
    if name == "commit":
        return n * (5 + u * (16 + 8 * channels)) if inline_values else n * (5 + u * 20)
    if name == "values":
        return n * u * (8 + 8 * channels)
    if name == "find":
        return n * (17 + READ_LINE)
    if name == "erase_mark":
        return n * (12 + READ_LINE + CAS64)
    if name == "erase_commit":
        return n * (1 + e * (4 + STORE))
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rho", type=float, default=0.5, choices=[0.1, 0.5, 0.99])
    ap.add_argument("--channels", type=int, default=8)
    ap.add_argument("--probe-group", type=int, default=4)
    ap.add_argument("--bucket-width", type=int, default=4)
    ap.add_argument("--max-load", type=float, default=0.5)
    ap.add_argument("--shape", choices=["tuned", "given"], default="tuned",
                    help="plain map: table shape from ash_autotune for the workload (tuned) or from "
                         "--probe-group/--bucket-width/--max-load (given)")
    ap.add_argument("--lds-dedup", action="store_true", help="drop block-local duplicates in LDS before probing")
    ap.add_argument("--sorted-keys", action="store_true",
                    help="insert the keys sorted (equal keys adjacent) instead of in random order")
    ap.add_argument("--cpu-sample", type=int, default=2_000_000,
                    help="positions of the workload the oracle runs for cpu_baseline (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy 128 MiB once with the library's streaming copy (reference kernel for byte counters)")
    ap.add_argument("--workload", default="plain",
                    choices=["plain", "batched", "voxelize", "served", "neighbors", "values", "large", "access",
                             "setup1", "construct", "ablation"],
                    help="plain: the headline 10M-key map; batched: 64 maps in one launch; voxelize: 5M points; "
                         "served: a Poisson request stream on a 2^25-capacity map")
    ap.add_argument("--requests", type=int, default=100_000, help="served: requests per run")
    ap.add_argument("--query-order", default="given", choices=["given", "morton"],
                    help="neighbors: query order (first appearance, or sorted by Z-order code)")
    ap.add_argument("--large-n", type=int, default=1_000_000_000, help="large: keys per insert and per find")
    ap.add_argument("--access-table-gib", type=float, default=16.0,
                    help="access: size of the large table (far beyond the 256 MB Infinity Cache)")
    ap.add_argument("--access-quick", action="store_true",
                    help="access: one launch per case (for counter runs under rocprofv3)")
    ap.add_argument("--neighbors-probe-group", type=int, default=1, help="neighbors: probe group of the map")
    ap.add_argument("--neighbors-bucket-width", type=int, default=4, help="neighbors: bucket width of the map")
    ap.add_argument("--served-max-load", type=float, default=0.5, help="served: max_load of the served map's table")
    # A served map sees many small batches whose kernels are latency-bound: one
    # lane per key probes all keys of a block at once (5.5 against 4.5 G
    # operations/s of burst capacity for g = 4, W = 4).
    ap.add_argument("--served-probe-group", type=int, default=1, help="served: probe group of the served map")
    ap.add_argument("--served-bucket-width", type=int, default=4, help="served: bucket width of the served map")
    ap.add_argument("--served-in-flight", type=int, default=4, help="served: device batches queued at once")
    ap.add_argument("--served-max-batch", type=int, default=1 << 22, help="served: positions per fused batch")
    ap.add_argument("--served-basis-mops", type=float, default=0.0,
                    help="served: offered loads are fractions of this rate (0: the plain path's mixed throughput)")
    ap.add_argument("--no-served", action="store_true", help="plain: skip the served-map leg of the bench line")
    ap.add_argument("--served-burst-only", action="store_true",
                    help="served: only the burst run (every request waiting), e.g. for a kernel trace of it")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU sharding is a design note only"}))
        sys.exit(2)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "voxelize":
        return bench_voxelize(args)
    if args.workload == "neighbors":
        return bench_neighbors(args)
    if args.workload == "values":
        return bench_values(args)
    if args.workload == "large":
        return bench_large(args)
    if args.workload == "access":
        return bench_access(args)
    if args.workload == "setup1":
        return bench_setup1(args)
    if args.workload == "construct":
        return bench_construct(args)
    if args.workload == "ablation":
        return bench_ablation(args)
    if args.workload == "served":
        return bench_served(args)

    import torch

    import paper_2110_00511_amd as ash
    import synth
    from paper_2110_00511_amd import _lib as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    d = synth.plain_large(rho=args.rho, channels=args.channels)
    if args.sorted_keys:
        order = np.lexsort(d["keys"].T[::-1])
        d["keys"], d["values"] = d["keys"][order], d["values"][order]
    n, nf, ne = len(d["keys"]), len(d["find_keys"]), len(d["erase_keys"])
    keys = torch.from_numpy(d["keys"]).cuda()
    vals = torch.from_numpy(d["values"]).cuda()
    fkeys = torch.from_numpy(d["find_keys"]).cuda()
    ekeys = torch.from_numpy(d["erase_keys"]).cuda()
    idx = torch.empty(n, dtype=torch.int32, device="cuda")
    mask = torch.empty(n, dtype=torch.uint8, device="cuda")
    fidx = torch.empty(nf, dtype=torch.int32, device="cuda")
    fmask = torch.empty(nf, dtype=torch.uint8, device="cuda")
    emask = torch.empty(ne, dtype=torch.uint8, device="cuda")
    tune_s = None
    if args.shape == "tuned":  # the shape the library's tuner picks for this workload on this GPU
        t0 = time.perf_counter()
        tun, _ = ash.autotune(d["capacity"], n, args.rho, 3, [(torch.float32, args.channels)])
        tune_s = time.perf_counter() - t0
        shape = (tun["probe_group"], tun["bucket_width"], round(float(tun["max_load"]), 4))
    else:
        shape = (args.probe_group, args.bucket_width, args.max_load)
    m = ash.HashMap(d["capacity"], 3, [(torch.float32, args.channels)], probe_group=shape[0],
                    bucket_width=shape[1], max_load=shape[2], lds_dedup=args.lds_dedup)
    lib = L.load()
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    vptr = (ctypes.c_void_p * 1)(vals.data_ptr())
    P = ctypes.c_void_p

    def step():
        L.check(lib.ash_clear(m._m, sp), "clear")
        L.check(lib.ash_insert(m._m, P(keys.data_ptr()), n, ctypes.cast(vptr, P), P(idx.data_ptr()),
                               P(mask.data_ptr()), sp), "insert")
        L.check(lib.ash_find(m._m, P(fkeys.data_ptr()), nf, P(fidx.data_ptr()), P(fmask.data_ptr()), None, sp),
                "find")
        L.check(lib.ash_erase(m._m, P(ekeys.data_ptr()), ne, P(emask.data_ptr()), sp), "erase")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    u = float(mask.sum().item()) / n
    dup = 1.0 - u  # fresh map each step: every non-new position repeats a new key of the batch
    eta = float(fmask.sum().item()) / nf
    e = float(emask.sum().item()) / ne
    assert m.device_status() == 0

    m.profile(True)
    m.profile_collect()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernels = m.profile_collect()
    m.profile(False)
    if args.copy_calibration:
        counter_calibration()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    inline = "values" not in kernels  # value rows copied inside the commit
    ops = n + nf + ne
    value = ops / (ms_per_step * 1e-3) / 1e6

    # Practical ceiling: a 1 GiB device-to-device copy (1 GiB read + 1 GiB
    # written per copy), timed after the steps on torch's stream.
    ca = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    cb = torch.empty_like(ca)
    cb.copy_(ca)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        cb.copy_(ca)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * (1 << 30) / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del ca, cb

    def avg_ms(name):
        return kernels[name][1] / kernels[name][0] if name in kernels else 0.0
    C = args.channels
    claim_name = next((k for k in kernels if k.startswith("claim")), "claim")
    ins_parts = [k for k in (claim_name, "sum_partials", "commit", "finalize", "values") if k in kernels]
    ins_ms = sum(avg_ms(k) for k in ins_parts)
    find_ms = avg_ms("find")
    erase_ms = avg_ms("erase_mark") + avg_ms("erase_commit")
    accounting = {"granule_B_measured": GRANULE_B, "copy_ceiling_GBps": round(copy_gbs, 1),
                  "note": "granule: each unavoidable random access counted as one DRAM granule g; payload: the "
                          "bytes the method touches; design: this implementation's per-kernel bytes"}
    rates = {}
    for op, cnt, ms in (("insert", n, ins_ms), ("find", nf, find_ms), ("erase", ne, erase_ms)):
        rate = cnt / (ms * 1e-3)
        rates[op] = rate
        ob = {g: op_bytes(op, g, u=u, eta=eta, e=e, C=C) for g in (GRANULE_B, 64)}
        entry = {"Mops": round(rate / 1e6, 1), "ms": round(ms, 4)}
        pay = ob[GRANULE_B]["payload"]
        entry["payload"] = {"B_per_op": round(pay, 1), "GBps": round(rate * pay / 1e9, 1),
                            "frac": round(rate * pay / 1e9 / HBM_PEAK_GBS, 4)}
        for g in (GRANULE_B, 64):
            gb = ob[g]["granule"]
            entry[f"granule_g{g}"] = {"B_per_op": round(gb, 1), "GBps": round(rate * gb / 1e9, 1),
                                      "frac": round(rate * gb / 1e9 / HBM_PEAK_GBS, 4)}
        if op == "find":  # the key is compared in its slot: no separate k^B read per hit
            gb = op_bytes("find_in_slot", GRANULE_B, eta=eta)["granule"]
            entry[f"granule_g{GRANULE_B}_key_in_slot"] = {
                "B_per_op": round(gb, 1), "GBps": round(rate * gb / 1e9, 1),
                "frac": round(rate * gb / 1e9 / HBM_PEAK_GBS, 4)}
        accounting[op] = entry
    accounting["insert"]["kernels"] = ins_parts

    per_kernel = {}
    for name, (launches, total) in kernels.items():
        avg = total / launches
        base = "claim" if name.startswith("claim") else name
        units = {"claim": n, "commit": n, "values": n, "find": nf, "erase_mark": ne, "erase_commit": ne}.get(base)
        b = kernel_bytes(base, units, u, dup, e, args.channels, inline) if units else None
        per_kernel[name] = {"launches_per_step": launches / args.steps, "avg_ms": round(avg, 4),
                            "design_GBps": round(b / (avg * 1e-3) / 1e9, 1) if b else None}
    # Roofline of the dominant operation, insert (its claim and commit take
    # over half the step): granule bytes per insert position x positions per
    # call / the summed average durations of its kernels.
    ins_bytes = op_bytes("insert", GRANULE_B, u=u, C=C)["granule"] * n
    achieved = ins_bytes / (ins_ms * 1e-3) / 1e9
    traffic = None
    mt = measured_traffic(args, shape)
    if mt is not None and all(k in mt for k in ins_parts):
        traffic = round(sum(mt[k] for k in ins_parts) / 1e9, 4)

    cpu = None
    if args.cpu_sample > 0:
        from oracle import OracleMap
        s = args.cpu_sample
        om = OracleMap(max(2 * s, 1), 3, [(np.float32, args.channels)])
        c0 = time.perf_counter()
        om.insert(d["keys"][:s], [d["values"][:s]])
        om.find(d["find_keys"][:s])
        om.erase(d["erase_keys"][: s // 2])
        c1 = time.perf_counter()
        cpu = {"value": round((s + s + s // 2) / (c1 - c0) / 1e6, 3), "unit": "Mops/s", "cores": 1,
               "of_cores": len(os.sched_getaffinity(0)), "host_cpus": os.cpu_count(), "cpu_model": cpu_model(),
               "kind": "oracle",
               "sample": f"insert first {s} keys, find first {s}, erase first {s // 2} of the same workload "
                         f"(std::map oracle, one thread of {len(os.sched_getaffinity(0))}, {c1 - c0:.1f} s)"}

    served = None
    if not args.no_served:
        served = served_leg(args)

    out = {
        "metric": "Mops/s insert+find (10M int32×3 keys) & %HBM peak; served p50/p99 latency",
        "value": round(value, 1),
        "unit": "Mops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"plain map at scale: insert {n} int32x3 keys (distinct ratio {args.rho}, "
                               f"f32x{args.channels} values), find {nf} (50% hits), erase {ne}",
                   "capacity": d["capacity"], "ops_per_step": ops, "probe_group": shape[0],
                   "bucket_width": shape[1], "max_load": shape[2], "shape_from": args.shape,
                   "autotune_s": None if tune_s is None else round(tune_s, 2), "lds_dedup": args.lds_dedup,
                   "sorted_keys": args.sorted_keys, "claim_variant": claim_name,
                   "measured": {"new_key_fraction": round(u, 4), "find_hit_rate": round(eta, 4),
                                "erase_win_fraction": round(e, 4)}},
        "roofline": {"bound": "hbm", "kernel": "insert (" + " + ".join(ins_parts) + ")", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_note": "L2-to-fabric bytes per call (FETCH_SIZE x2 + WRITE_SIZE, Infinity Cache "
                                     "hits included), from counter runs of these kernel sources",
                     "accounting": "granule", "granule_B": GRANULE_B,
                     "bytes_per_op": round(ins_bytes / n, 1), "units_per_launch": n,
                     "frac_g64": round(op_bytes("insert", 64, u=u, C=C)["granule"] * n / (ins_ms * 1e-3) / 1e9
                                       / HBM_PEAK_GBS, 4)},
        "kernels": per_kernel,
        "accounting": accounting,
        "cpu_baseline": cpu,
        "served": served,
    }
    print(json.dumps(out), flush=True)


def counter_calibration():
    """A kernel of known traffic for counter runs: the library's streaming
    copy of a 256 MiB buffer's first half onto its second (128 MiB read,
    128 MiB written).  (torch's device-to-device copy may run on a copy
    engine, which the counters do not see.)"""
    import torch

    from paper_2110_00511_amd import _lib as L
    lib = L.load()
    cal = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    cms = ctypes.c_double()
    L.check(lib.ash_access_bench(L.ASH_ACC_STREAM_COPY, ctypes.c_void_p(cal.data_ptr()), cal.numel(), 16, 0, 1,
                                 ctypes.byref(cms), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
            "calibration copy")
    torch.cuda.synchronize()
    del cal


def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def batched_grid(lib, sp):
    """Blocks of the persistent batched launch (int32x3 keys) per kernel
    build: the count the device ran at once and the occupancy the runtime
    reported."""
    from paper_2110_00511_amd import _lib as L
    out = {}
    for narrow, name in ((1, "lane_w2_w4_build"), (0, "general_build")):
        blocks, reported = ctypes.c_int64(0), ctypes.c_int64(0)
        L.check(lib.ash_batched_grid(3, narrow, ctypes.byref(blocks), ctypes.byref(reported), sp), "batched grid")
        out[name] = {"blocks": blocks.value, "reported": reported.value}
    return out


def bench_batched(args):
    """64 independent maps (distinct counts log-uniform in [1e3, 1e6], f32x8
    values): the inserts and finds of all maps in one persistent launch,
    called through the C ABI with descriptors and outputs built once, beside
    the same work op by op through the single-map path.  Each path gets the
    table shapes its own autotuner picks (ash_autotune_batched for the fused
    launch, ash_autotune for the single-map path).  Every map is cleared
    before each trial, outside the timed call (the figures with the clears
    inside are reported too)."""
    import torch

    import paper_2110_00511_amd as ash
    import synth
    from paper_2110_00511_amd import _lib as L

    torch.cuda.set_device(0)
    work = synth.batched()
    lib = L.load()
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = ctypes.c_void_p
    keep = []

    def build(batched_tuning, grid=None):
        t0 = time.perf_counter()
        maps = []
        for w in work:
            tun, _ = ash.autotune(w["capacity"], len(w["keys"]), 0.5, 3, [(torch.float32, 8)], batched=batched_tuning,
                                  grid=grid)
            maps.append((ash.HashMap(w["capacity"], 3, [(torch.float32, 8)], **tun), tun))
        tune_s = time.perf_counter() - t0
        arr = (L.AshBatchOp * len(work))()
        for i, (w, (m, _)) in enumerate(zip(work, maps)):
            ik = torch.from_numpy(w["keys"]).cuda()
            iv = torch.from_numpy(w["values"]).cuda()
            fk = torch.from_numpy(w["find_keys"]).cuda()
            ni, nf = ik.shape[0], fk.shape[0]
            outs = [torch.empty(ni, dtype=torch.int32, device="cuda"),
                    torch.empty(ni, dtype=torch.uint8, device="cuda"),
                    torch.empty(nf, dtype=torch.int32, device="cuda"),
                    torch.empty(nf, dtype=torch.uint8, device="cuda")]
            vin = (P * 1)(iv.data_ptr())
            keep.extend([ik, iv, fk, outs, vin])
            arr[i] = L.AshBatchOp(m._m, ik.data_ptr(), ni, ctypes.cast(vin, P), outs[0].data_ptr(),
                                  outs[1].data_ptr(), fk.data_ptr(), nf, None, outs[2].data_ptr(), outs[3].data_ptr())
        shapes = {}
        for _, t in maps:
            k = f"g{t['probe_group']}_w{t['bucket_width']}_lf{t['max_load']:.2f}"
            shapes[k] = shapes.get(k, 0) + 1
        return maps, arr, shapes, tune_s

    maps_f, arr_f, shapes_f, tune_f = build(True)
    maps_p, arr_p, shapes_p, tune_p = build(False)
    # the grid the batched workload states: W {4, 8, 16, 32} x max load {0.5,
    # 0.7, 0.85} x probe group {8, 16, 64}, each point timed in the persistent launch
    stated = ([4, 8, 16, 32], [8, 16, 64], [0.5, 0.7, 0.85])
    maps_s, arr_s, shapes_s, tune_s = build(True, grid=stated)
    n_ops = sum(len(w["keys"]) + len(w["find_keys"]) for w in work)

    def clear_all(maps):
        for m, _ in maps:
            L.check(lib.ash_clear(m._m, sp), "clear")

    def run(arr, fused):
        L.check(lib.ash_batched(arr, len(work), 1 if fused else 0, sp), "ash_batched")

    def timed_hot(maps, arr, fused):
        """Mean ms of the batched call alone; the clears run untimed before each trial."""
        for _ in range(args.warmup):
            clear_all(maps)
            run(arr, fused)
        total = 0.0
        for _ in range(args.steps):
            clear_all(maps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run(arr, fused)
            torch.cuda.synchronize()
            total += time.perf_counter() - t0
        return total * 1e3 / args.steps

    ms_f = timed_hot(maps_f, arr_f, True)
    ms_p = timed_hot(maps_p, arr_p, False)
    ms_s = timed_hot(maps_s, arr_s, True)
    ms_fc = _timed(lambda: (clear_all(maps_f), run(arr_f, True)), args.steps, args.warmup)
    ms_pc = _timed(lambda: (clear_all(maps_p), run(arr_p, False)), args.steps, args.warmup)
    print(json.dumps({
        "metric": "Mops/s insert+find, 64 batched maps in one persistent launch", "value": round(n_ops / ms_f / 1e3, 1),
        "unit": "Mops/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_f, 4),
        "higher_is_better": True, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"64 maps, distinct counts log-uniform in [1e3, 1e6], {n_ops} key ops per step "
                               "(insert 2u then find 2u per map), f32x8 values; maps cleared untimed before "
                               "each step",
                   "tuned_shapes": shapes_f, "autotune_s": round(tune_f, 2)},
        "plain_path": {"ms_per_step": round(ms_p, 4), "value": round(n_ops / ms_p / 1e3, 1), "unit": "Mops/s",
                       "tuned_shapes": shapes_p, "autotune_s": round(tune_p, 2)},
        "speedup_vs_plain": round(ms_p / ms_f, 3),
        "stated_grid": {"grid": {"bucket_width": stated[0], "probe_group": stated[1], "max_load": stated[2]},
                        "ms_per_step": round(ms_s, 4), "value": round(n_ops / ms_s / 1e3, 1), "unit": "Mops/s",
                        "tuned_shapes": shapes_s, "autotune_s": round(tune_s, 2)},
        "fallbacks": int(lib.ash_batched_fallbacks()),
        "resident_blocks": batched_grid(lib, sp),
        "with_clears": {"fused_ms": round(ms_fc, 4), "plain_ms": round(ms_pc, 4),
                        "fused_Mops": round(n_ops / ms_fc / 1e3, 1), "plain_Mops": round(n_ops / ms_pc / 1e3, 1)}}),
          flush=True)


def bench_voxelize(args):
    """5M surface points, voxel 5 mm (and 1, 2, 5 cm): Mpoints/s of ash_voxelize."""
    import torch

    import paper_2110_00511_amd as ash
    import synth

    torch.cuda.set_device(0)
    pts = torch.from_numpy(synth.points()).cuda()
    n = pts.shape[0]
    out = {}
    for v in (0.005, 0.01, 0.02, 0.05):
        res = {}

        def step():
            res["r"] = ash.voxelize(pts, v)

        ms = _timed(step, args.steps, args.warmup)
        out[f"{v * 100:g}cm"] = {"ms": round(ms, 4), "Mpoints_per_s": round(n / ms / 1e3, 1),
                                 "voxels": int(res["r"][1].shape[0])}
    ms0 = out["0.5cm"]["ms"]
    cpu = None
    if args.cpu_sample > 0:
        from oracle import oracle_voxelize
        s = min(args.cpu_sample, n)
        pnp = synth.points()[:s]
        c0 = time.perf_counter()
        oracle_voxelize(pnp, 0.005)
        c1 = time.perf_counter()
        cpu = {"value": round(s / (c1 - c0) / 1e6, 3), "unit": "Mpoints/s", "cores": 1, "kind": "oracle",
               "sample": f"first {s} points at 5 mm ({c1 - c0:.1f} s)"}
    # Roofline of one whole call (its kernels are launched back to back on one
    # stream): algorithmic bytes per point with u = voxels / points --
    # claim: point 12 + window line + u * CAS + slot 4; commit: slot 4 +
    # lost 1 + point id 4 + u * (voxel key 12 + count 4 [+ slot store 32 when
    # u <= 1/2, the voxel's id written into its slot]); resolve: slot 4 +
    # (1 - u) * (slot line [+ the first point's id line when u > 1/2] + count
    # atomic + point id 4); fills: the 16 B slots of a table at load 0.5
    # (32 B per point) and 1 B per point of scratch.
    u = out["0.5cm"]["voxels"] / n
    publish = u <= 0.5
    per_point = (12 + READ_LINE + u * CAS64 + 4) + (4 + 1 + 4 + u * (12 + 4 + (STORE if publish else 0))) \
        + (4 + (1 - u) * (READ_LINE + (0 if publish else READ_LINE) + ATOM32 + 4)) + (32 + 1)
    achieved = per_point * n / (ms0 / 1e3) / 1e9
    print(json.dumps({
        "metric": "Mpoints/s voxelization (5M points, 5 mm voxels)", "value": round(n / ms0 / 1e3, 1),
        "unit": "Mpoints/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms0,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n} points on 20 random spheres/planes in a 10 m box, sigma 1 cm", "sweep": out},
        "roofline": {"bound": "hbm", "kernel": "voxelize (one whole call)", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "algorithmic_bytes_per_point": round(per_point, 1)},
        "cpu_baseline": cpu}), flush=True)


def bench_values(args):
    """Setup 1's value-size sweep (Sec. 5.1): 1M int32x3 keys (distinct ratio
    0.99) with f32 x 2^j value rows, j = 0..12 (4 B to 16 KB), capacity = the
    number of keys.  Per size: insert into a cleared map, then a 50%-hit find
    that gathers the hits' rows.  Rows under 64 B are copied inside the commit
    and the find; longer ones by the separate row pass after the commit.
    Value rows are drawn on the device from a seeded generator."""
    import torch

    import paper_2110_00511_amd as ash
    import synth
    from paper_2110_00511_amd import _lib as L

    torch.cuda.set_device(0)
    d = synth.value_sweep()
    n, nf = len(d["keys"]), len(d["find_keys"])
    keys = torch.from_numpy(d["keys"]).cuda()
    fkeys = torch.from_numpy(d["find_keys"]).cuda()
    idx = torch.empty(n, dtype=torch.int32, device="cuda")
    mask = torch.empty(n, dtype=torch.uint8, device="cuda")
    fidx = torch.empty(nf, dtype=torch.int32, device="cuda")
    fmask = torch.empty(nf, dtype=torch.uint8, device="cuda")
    lib = L.load()
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = ctypes.c_void_p
    gen = torch.Generator(device="cuda")
    gen.manual_seed(8)
    sweep = {}
    for j in range(0, 13):
        ch = 1 << j
        m = ash.HashMap(n, 3, [(torch.float32, ch)])
        vals = torch.randn((n, ch), dtype=torch.float32, device="cuda", generator=gen)
        outv = torch.empty((nf, ch), dtype=torch.float32, device="cuda")
        vptr = (ctypes.c_void_p * 1)(vals.data_ptr())
        optr = (ctypes.c_void_p * 1)(outv.data_ptr())

        def ins():
            L.check(lib.ash_clear(m._m, sp), "clear")
            L.check(lib.ash_insert(m._m, P(keys.data_ptr()), n, ctypes.cast(vptr, P), P(idx.data_ptr()),
                                   P(mask.data_ptr()), sp), "insert")

        def fnd():
            L.check(lib.ash_find(m._m, P(fkeys.data_ptr()), nf, P(fidx.data_ptr()), P(fmask.data_ptr()),
                                 ctypes.cast(optr, P), sp), "find")
        steps = max(1, args.steps // (1 if j < 10 else 2))
        ins()
        m.profile(True)
        m.profile_collect()
        t_ins = _timed(ins, steps, 1)
        kern = {k: v[1] / v[0] for k, v in m.profile_collect().items()}
        t_fnd = _timed(fnd, steps, 1)
        kern_f = {k: v[1] / v[0] for k, v in m.profile_collect().items()}
        m.profile(False)
        assert m.device_status() == 0
        u = int(mask.sum().item())
        hits = int(fmask.sum().item())
        row = 4 * ch
        # value bytes moved: each inserted row read from the batch and written to v^B, each hit row read and written
        ins_gb = 2.0 * u * row / 1e9
        fnd_gb = 2.0 * hits * row / 1e9
        sweep[f"f32x{ch}"] = {
            "row_bytes": row, "insert_ms": round(t_ins, 4), "find_ms": round(t_fnd, 4),
            "insert_Mops": round(n / t_ins / 1e3, 1), "find_Mops": round(nf / t_fnd / 1e3, 1),
            "insert_value_GBps": round(ins_gb / t_ins * 1e3, 1), "find_value_GBps": round(fnd_gb / t_fnd * 1e3, 1),
            "kernel_ms": {k: round(v, 4) for k, v in {**kern, **{"find": kern_f.get("find", 0.0)}}.items()},
            "new_keys": u, "hits": hits}
        del m, vals, outv
        torch.cuda.empty_cache()
    top = sweep["f32x4096"]
    # roofline of the dominant kernel at 16 KB rows: the separate row pass reads and writes every inserted row
    vk = top["kernel_ms"]["values"]
    achieved = (top["new_keys"] * (2 * top["row_bytes"] + 8)) / (vk / 1e3) / 1e9
    print(json.dumps({
        "metric": "value-row GB/s moved by insert (1M keys, f32x4096 rows); Setup 1 sweep f32x1..4096",
        "value": top["insert_value_GBps"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": top["insert_ms"], "higher_is_better": True, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"{n} int32x3 keys (distinct ratio 0.99), capacity {n}, f32 x 2^j rows; "
                               f"{nf} finds (half hits) gathering rows", "sweep": sweep},
        "roofline": {"bound": "hbm", "kernel": "values", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes_per_row": 2 * top["row_bytes"] + 8, "kernel_ms": vk},
        "cpu_baseline": None}), flush=True)


def _event_ms(fn, trials):
    """Median GPU time of fn() between two events on torch's current stream
    (the library launches on that stream), one untimed call first."""
    import torch
    fn()
    ts = []
    for _ in range(trials):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def bench_setup1(args):
    """Setup 1 of Sec. 5.1: int32x3 keys, f32 x 2^j values (j = 0..12),
    capacities c = 10^3..10^6 with c input keys, distinct ratios 0.1 and
    0.99.  Per point: insert into a cleared map, activate into a cleared
    map (keys only: the paper reports its time flat in the value size), and
    a 50%-hit find that gathers the hits' rows; each the median GPU time of
    10 calls (the map is cleared before each insert or activate, outside the
    timed call)."""
    import torch

    import paper_2110_00511_amd as ash
    import synth
    from paper_2110_00511_amd import _lib as L

    torch.cuda.set_device(0)
    lib = L.load()
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = ctypes.c_void_p
    gen = torch.Generator(device="cuda")
    gen.manual_seed(10)
    grid = {}
    for c in (1_000, 10_000, 100_000, 1_000_000):
        for rho in (0.1, 0.99):
            d = synth.setup1(c, rho)
            keys = torch.from_numpy(d["keys"]).cuda()
            fkeys = torch.from_numpy(d["find_keys"]).cuda()
            idx = torch.empty(c, dtype=torch.int32, device="cuda")
            mask = torch.empty(c, dtype=torch.uint8, device="cuda")
            fidx = torch.empty(c, dtype=torch.int32, device="cuda")
            fmask = torch.empty(c, dtype=torch.uint8, device="cuda")
            row = {}
            for j in range(13):
                ch = 1 << j
                m = ash.HashMap(c, 3, [(torch.float32, ch)])
                vals = torch.randn((c, ch), dtype=torch.float32, device="cuda", generator=gen)
                outv = torch.empty((c, ch), dtype=torch.float32, device="cuda")
                vptr = (ctypes.c_void_p * 1)(vals.data_ptr())
                optr = (ctypes.c_void_p * 1)(outv.data_ptr())
                times = {}
                for op in ("insert", "activate"):
                    def one(op=op):
                        if op == "insert":
                            L.check(lib.ash_insert(m._m, P(keys.data_ptr()), c, ctypes.cast(vptr, P),
                                                   P(idx.data_ptr()), P(mask.data_ptr()), sp), "insert")
                        else:
                            L.check(lib.ash_activate(m._m, P(keys.data_ptr()), c, P(idx.data_ptr()),
                                                     P(mask.data_ptr()), sp), "activate")
                    ts = []
                    for _ in range(11):
                        L.check(lib.ash_clear(m._m, sp), "clear")
                        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        a.record()
                        one()
                        b.record()
                        b.synchronize()
                        ts.append(a.elapsed_time(b))
                    times[op] = float(np.median(ts[1:]))
                L.check(lib.ash_clear(m._m, sp), "clear")
                L.check(lib.ash_insert(m._m, P(keys.data_ptr()), c, ctypes.cast(vptr, P), P(idx.data_ptr()),
                                       P(mask.data_ptr()), sp), "insert")
                times["find"] = _event_ms(lambda: L.check(lib.ash_find(
                    m._m, P(fkeys.data_ptr()), c, P(fidx.data_ptr()), P(fmask.data_ptr()), ctypes.cast(optr, P),
                    sp), "find"), 10)
                assert m.device_status() == 0
                row[str(4 * ch)] = {k: round(v * 1e3, 2) for k, v in times.items()}  # microseconds
                m.close()
                del vals, outv
            u = int(mask.sum().item())
            grid[f"c={c},rho={rho}"] = {"distinct": u, "us_by_row_bytes": row}
            print(f"# setup1 c={c} rho={rho}: {row}", flush=True)
            torch.cuda.empty_cache()
    flat = {k: round(v["us_by_row_bytes"]["16384"]["activate"] / v["us_by_row_bytes"]["4"]["activate"], 3)
            for k, v in grid.items()}
    grow = {k: round(v["us_by_row_bytes"]["16384"]["insert"] / v["us_by_row_bytes"]["4"]["insert"], 3)
            for k, v in grid.items()}
    top = grid["c=1000000,rho=0.99"]["us_by_row_bytes"]["4"]
    print(json.dumps({
        "metric": "Setup 1 grid: insert / activate / find microseconds (int32x3 keys, f32 x 2^j values)",
        "value": round(1_000_000 / top["insert"], 1), "unit": "Mops/s (insert, c = 10^6, rho 0.99, 4 B rows)",
        "n_gpus": 1, "higher_is_better": True, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "c in {1e3, 1e4, 1e5, 1e6} keys (capacity c), rho in {0.1, 0.99}, f32 x 2^j "
                               "values j = 0..12; median GPU time of 10 calls per point"},
        "activate_16KB_over_4B": flat, "insert_16KB_over_4B": grow, "grid": grid, "cpu_baseline": None}),
        flush=True)


def bench_construct(args):
    """Construction time (Sec. 5.2 reports under 1 ms for c = 10^3..10^6):
    ash_create of an int32x3 -> f32 map of capacity c, which allocates the
    table, key, value, heap and owner buffers, fills the table, writes the
    heap 0..c-1 and synchronizes; then ash_destroy.  Host clock around each
    call, median of 10 after one warm-up, with torch's caching allocator
    (blocks reused after the first create) and with plain hipMalloc."""
    import torch

    from paper_2110_00511_amd import _lib as L

    torch.cuda.set_device(0)
    lib = L.load()
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    alloc = L.TorchAllocator("cuda")
    dts = (ctypes.c_int * 1)(L.ASH_F32)
    els = (ctypes.c_int64 * 1)(1)
    res = {}
    for c in (1_000, 10_000, 100_000, 1_000_000, 10_000_000):
        row = {}
        for name, a in (("torch_allocator", ctypes.byref(alloc.struct)), ("hipMalloc", None)):
            tc, td = [], []
            for rep in range(11):
                out = ctypes.c_void_p()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                L.check(lib.ash_create(c, 3, 1, ctypes.cast(dts, ctypes.c_void_p), ctypes.cast(els, ctypes.c_void_p),
                                       a, None, sp, ctypes.byref(out)), "create")
                t1 = time.perf_counter()
                L.check(lib.ash_destroy(out), "destroy")
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                if rep:
                    tc.append(t1 - t0)
                    td.append(t2 - t1)
            row[name] = {"create_ms": round(float(np.median(tc)) * 1e3, 3),
                         "destroy_ms": round(float(np.median(td)) * 1e3, 3)}
        res[str(c)] = row
        print(f"# construct c={c}: {row}", flush=True)
    top = res["1000000"]["torch_allocator"]["create_ms"]
    print(json.dumps({
        "metric": "map construction time (ash_create, synchronized)", "value": top,
        "unit": "ms at c = 10^6 (torch caching allocator)", "n_gpus": 1, "higher_is_better": False,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": "int32x3 -> f32 map, capacity 10^3..10^7, default tuning; median of 10"},
        "results": res, "cpu_baseline": None}), flush=True)


def bench_ablation(args):
    """Backend ablation (Sec. 5.2 and 5.3): the separate-chaining backend of
    include/ash_slab.h (slab lists, index delegates, three-pass insertion)
    beside the product's open addressing, on the same inputs.
    Setup 2: scalar int32 keys -> f32, c = 10^3..10^6 keys into capacity c,
    distinct ratio 0.1 / 0.5 / 0.99.  Setup 1 shape: int32x3 keys, c = 10^6,
    distinct ratio 0.1 / 0.99, f32 x {1, 8, 64, 512} rows.  Per point the
    median GPU time of 10 calls: insert into a cleared map, then a 50%-hit
    find that gathers rows."""
    import torch

    import paper_2110_00511_amd as ash
    import synth
    from paper_2110_00511_amd import _lib as L
    from paper_2110_00511_amd.ablation import SlabMap

    torch.cuda.set_device(0)
    lib = L.load()
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = ctypes.c_void_p
    gen = torch.Generator(device="cuda")
    gen.manual_seed(12)

    def one_point(kd, c, keys_np, fk_np, ch):
        keys = torch.from_numpy(keys_np).cuda()
        fkeys = torch.from_numpy(fk_np).cuda()
        vals = torch.randn((c, ch), dtype=torch.float32, device="cuda", generator=gen)
        idx = torch.empty(c, dtype=torch.int32, device="cuda")
        mask = torch.empty(c, dtype=torch.uint8, device="cuda")
        fidx = torch.empty(c, dtype=torch.int32, device="cuda")
        fmask = torch.empty(c, dtype=torch.uint8, device="cuda")
        outv = torch.empty((c, ch), dtype=torch.float32, device="cuda")
        res = {}
        # product: open addressing
        m = ash.HashMap(c, kd, [(torch.float32, ch)])
        vptr = (ctypes.c_void_p * 1)(vals.data_ptr())
        optr = (ctypes.c_void_p * 1)(outv.data_ptr())
        ts = []
        for _ in range(11):
            L.check(lib.ash_clear(m._m, sp), "clear")
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            L.check(lib.ash_insert(m._m, P(keys.data_ptr()), c, ctypes.cast(vptr, P), P(idx.data_ptr()),
                                   P(mask.data_ptr()), sp), "insert")
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        u = int(mask.sum().item())
        fnd = _event_ms(lambda: L.check(lib.ash_find(m._m, P(fkeys.data_ptr()), c, P(fidx.data_ptr()),
                                                     P(fmask.data_ptr()), ctypes.cast(optr, P), sp), "find"), 10)
        res["open_addressing"] = {"insert_us": round(float(np.median(ts[1:])) * 1e3, 2), "find_us": round(fnd * 1e3, 2)}
        m.close()
        # ablation: separate chaining
        s = SlabMap(c, kd, 4 * ch)
        ts = []
        for _ in range(11):
            L.check(lib.ash_slab_clear(s._m, sp), "slab clear")
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            L.check(lib.ash_slab_insert(s._m, P(keys.data_ptr()), c, P(vals.data_ptr()), P(idx.data_ptr()),
                                        P(mask.data_ptr()), sp), "slab insert")
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        assert int(mask.sum().item()) == u  # the same keys were inserted
        fnd = _event_ms(lambda: L.check(lib.ash_slab_find(s._m, P(fkeys.data_ptr()), c, P(fidx.data_ptr()),
                                                          P(fmask.data_ptr()), P(outv.data_ptr()), sp),
                                        "slab find"), 10)
        res["separate_chaining"] = {"insert_us": round(float(np.median(ts[1:])) * 1e3, 2),
                                    "find_us": round(fnd * 1e3, 2)}
        s.close()
        res["distinct"] = u
        return res

    setup2 = {}
    for c in (1_000, 10_000, 100_000, 1_000_000):
        for rho in (0.1, 0.5, 0.99):
            d = synth.setup2(c, rho)
            setup2[f"c={c},rho={rho}"] = one_point(1, c, d["keys"], d["find_keys"], 1)
            print(f"# ablation setup2 c={c} rho={rho}: {setup2[f'c={c},rho={rho}']}", flush=True)
    setup1 = {}
    for rho in (0.1, 0.99):
        d = synth.setup1(1_000_000, rho)
        for ch in (1, 8, 64, 512):
            setup1[f"rho={rho},row={4 * ch}B"] = one_point(3, 1_000_000, d["keys"], d["find_keys"], ch)
            print(f"# ablation setup1 rho={rho} row={4 * ch}: {setup1[f'rho={rho},row={4 * ch}B']}", flush=True)
    top = setup1["rho=0.99,row=4B"]
    print(json.dumps({
        "metric": "backend ablation: insert / find microseconds, open addressing vs separate chaining",
        "value": round(top["separate_chaining"]["insert_us"] / top["open_addressing"]["insert_us"], 3),
        "unit": "separate-chaining / open-addressing insert time (int32x3, 10^6 keys, rho 0.99, 4 B rows)",
        "n_gpus": 1, "higher_is_better": False, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "Setup 2 (scalar int32 -> f32, c = 1e3..1e6, rho 0.1/0.5/0.99) and int32x3 keys "
                               "at c = 1e6 with f32 x {1, 8, 64, 512} rows; median of 10 calls"},
        "setup2": setup2, "setup1_rows": setup1, "cpu_baseline": None}), flush=True)


def bench_large(args):
    """A hash set far beyond the caches: n int32x3 keys (default 1e9, distinct
    ratio ~0.5, drawn on the device from a seeded generator) inserted into a
    cleared map of capacity 0.65 n (max load 0.5), then n finds, half hits.
    Shows how insert and find rates hold up as the table grows to tens of GB."""
    import torch

    import paper_2110_00511_amd as ash

    torch.cuda.set_device(0)
    n = args.large_n
    gen = torch.Generator(device="cuda")
    gen.manual_seed(9)
    side = int(round((n / 1.5936) ** (1 / 3)))  # n draws from side^3 cells: ~0.5 distinct
    keys = torch.randint(0, side, (n, 3), dtype=torch.int32, device="cuda", generator=gen)
    fk = keys[torch.randint(0, n, (n,), device="cuda", generator=gen)]
    fk[n // 2:] += side  # the second half misses
    m = ash.HashMap(int(n * 0.65), 3, [], probe_group=args.probe_group, bucket_width=args.bucket_width,
                    max_load=args.max_load)
    from paper_2110_00511_amd import _lib as L
    lib = L.load()
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = ctypes.c_void_p
    idx = torch.empty(n, dtype=torch.int32, device="cuda")
    mask = torch.empty(n, dtype=torch.uint8, device="cuda")
    fidx = torch.empty(n, dtype=torch.int32, device="cuda")
    fm = torch.empty(n, dtype=torch.uint8, device="cuda")
    t_ins, t_fnd = [], []
    for step in range(args.warmup + args.steps):
        L.check(lib.ash_clear(m._m, sp), "clear")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.check(lib.ash_insert(m._m, P(keys.data_ptr()), n, None, P(idx.data_ptr()), P(mask.data_ptr()), sp), "insert")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.check(lib.ash_find(m._m, P(fk.data_ptr()), n, P(fidx.data_ptr()), P(fm.data_ptr()), None, sp), "find")
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if step >= args.warmup:
            t_ins.append(t1 - t0)
            t_fnd.append(t2 - t1)
    ti, tf = sum(t_ins) / len(t_ins), sum(t_fnd) / len(t_fnd)
    st = m.stats()
    assert m.device_status() == 0
    print(json.dumps({
        "metric": "Mops/s insert+find on a large hash set", "value": round(2 * n / (ti + tf) / 1e6, 1),
        "unit": "Mops/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round((ti + tf) * 1e3, 2), "higher_is_better": True, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"{n} int32x3 keys (distinct ratio ~0.5), hash set, then {n} finds (half hits)",
                   "distinct": st["size"], "slots": st["slots"], "table_GB": round(st["slots"] * 16 / 1e9, 1),
                   "insert_ms": round(ti * 1e3, 2), "insert_Mops": round(n / ti / 1e6, 1),
                   "find_ms": round(tf * 1e3, 2), "find_Mops": round(n / tf / 1e6, 1),
                   "hit_rate": round(float(fm.float().mean().item()), 4)},
        "cpu_baseline": None}), flush=True)


def bench_access(args):
    """Cost of one random access to a table far beyond every cache (16 GiB by
    default) and to a table of the 10M-key map's size (320 MiB, a little
    beyond the 256 MB Infinity Cache): random reads of 4..256 B, random
    stores, device-scope CAS and atomic min, and streaming read and copy of
    the table for reference.  Reads of A >= 16 B are made by A / 16 adjacent
    lanes (a probe group reading a window).

    The DRAM granule g of a small random read follows from timing alone:
    random reads of 256 B move whole lines and no byte they do not need, so
    their byte rate B256 is the rate at which the memory system serves random
    lines; a 16 B read that costs g bytes then runs at B256 / g reads/s, and
    g16 = B256 / R16.  rocprofv3 FETCH_SIZE / WRITE_SIZE of the same kernels
    (see the access profile summary) give the bytes directly."""
    import torch

    from paper_2110_00511_amd import _lib as L

    torch.cuda.set_device(0)
    lib = L.load()
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    reps = 1 if args.access_quick else 3
    tables = [("large", int(args.access_table_gib * (1 << 30)) // 256 * 256), ("map10M", 320 << 20)]
    n_read = 1 << 27
    n_store = 1 << 26
    n_atomic = 1 << 26
    cases = [("read", L.ASH_ACC_READ, a, n_read) for a in (4, 16, 32, 64, 128, 256)]
    cases += [("store", L.ASH_ACC_STORE, a, n_store) for a in (8, 16, 64, 128)]
    cases += [("cas64", L.ASH_ACC_CAS64, 8, n_atomic), ("min32", L.ASH_ACC_MIN32, 4, n_atomic),
              ("stream_read", L.ASH_ACC_STREAM_READ, 16, 0), ("stream_copy", L.ASH_ACC_STREAM_COPY, 16, 0)]
    results = {}
    for tname, tbytes in tables:
        buf = torch.zeros(tbytes, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        res = {}
        for kname, kind, abytes, n in cases:
            ms_all = []
            for r in range(reps + (0 if args.access_quick else 1)):
                ms = ctypes.c_double()
                L.check(lib.ash_access_bench(kind, ctypes.c_void_p(buf.data_ptr()), tbytes, abytes, n, 1234 + r,
                                             ctypes.byref(ms), sp), f"access {kname} {abytes}")
                ms_all.append(ms.value)
            ms = min(ms_all[-reps:])
            key = f"{kname}_{abytes}" if kname in ("read", "store") else kname
            if kname == "stream_read":
                res[key] = {"ms": round(ms, 4), "GBps": round(tbytes / (ms * 1e-3) / 1e9, 1)}
            elif kname == "stream_copy":
                res[key] = {"ms": round(ms, 4), "GBps_read_plus_write": round(tbytes / (ms * 1e-3) / 1e9, 1)}
            else:
                rate = n / (ms * 1e-3)
                res[key] = {"ms": round(ms, 4), "n": n, "G_per_s": round(rate / 1e9, 2),
                            "GBps_at_access_size": round(rate * abytes / 1e9, 1)}
            print(f"# access {tname} {key}: {res[key]}", flush=True)
        b256 = res["read_256"]["G_per_s"] * 256
        res["granule_from_timing_B"] = {f"read_{a}": round(b256 / res[f"read_{a}"]["G_per_s"], 1)
                                        for a in (4, 16, 32, 64, 128)}
        results[tname] = {"table_bytes": tbytes, **res}
        del buf
        torch.cuda.empty_cache()
    g16 = results["large"]["granule_from_timing_B"]["read_16"]
    print(json.dumps({
        "metric": "random access cost on MI355X (instrumentation)", "value": g16, "unit": "B per random 16 B read",
        "n_gpus": 1, "higher_is_better": False, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "random reads/stores/atomics at hashed addresses; streaming read and copy"},
        "results": results}), flush=True)


def morton3(keys):
    """Z-order code of int32x3 keys (21 bits per word after a shift to
    non-negative), for ordering queries so neighbors of nearby cells are
    looked up close in time."""
    k = (keys - keys.min(axis=0)).astype(np.uint64) & np.uint64((1 << 21) - 1)
    code = np.zeros(len(keys), np.uint64)
    for b in range(21):
        for d in range(3):
            code |= ((k[:, d] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + d)
    return code


def bench_neighbors(args):
    """Neighbor search (Listing 3 of Sec. 6.2.4): the 27 radius-1 neighbors of
    every distinct 5 mm lattice cell of the 5M-point surface cloud (4.8M
    cells, the key set and the query set), one ash_find_offsets call per step.
    Beside it: the 1-ring (6) and 1-cube (8) neighborhoods of Sec. 6.3 and the
    intersection of the cells with a copy shifted by one cell (Sec. 6.4)."""
    import torch

    import paper_2110_00511_amd as ash
    import synth
    from paper_2110_00511_amd import _lib as L

    torch.cuda.set_device(0)
    keys_np = synth.surface_keys()
    if args.query_order == "morton":
        keys_np = keys_np[np.argsort(morton3(keys_np), kind="stable")]
    n = len(keys_np)
    keys = torch.from_numpy(keys_np).cuda()
    m = ash.HashMap(n, 3, probe_group=args.neighbors_probe_group, bucket_width=args.neighbors_bucket_width,
                    max_load=args.max_load)
    m.insert(keys)
    lib = L.load()
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = ctypes.c_void_p
    outs = {}

    def run(kind, radius, steps, warmup, profile=False):
        off = ash.neighbor_offsets(kind, radius)
        k = off.shape[0]
        idx = torch.empty((n, k), dtype=torch.int32, device="cuda")
        mask = torch.empty((n, k), dtype=torch.uint8, device="cuda")

        def step():
            L.check(lib.ash_find_offsets(m._m, P(keys.data_ptr()), n, P(off.data_ptr()), k, P(idx.data_ptr()),
                                         P(mask.data_ptr()), sp), "find_offsets")
        if profile:
            for _ in range(warmup):
                step()
            m.profile(True)
            m.profile_collect()
            ms = _timed(step, steps, 0)
            launches, total = m.profile_collect()["find_offsets"]
            m.profile(False)
            outs["kernel_ms"] = total / launches
        else:
            ms = _timed(step, steps, warmup)
        return k, ms, float(mask.float().mean().item())

    k, ms, hit = run("radius", 1, args.steps, args.warmup, profile=True)
    if args.copy_calibration:
        counter_calibration()
    sweep = {"radius1": {"offsets": k, "ms": round(ms, 4), "Mlookups_per_s": round(n * k / ms / 1e3, 1),
                         "hit_rate": round(hit, 4)}}
    for kind, r in (("ring", 1), ("cube", 1), ("radius", 2)):
        kk, mss, h = run(kind, r, max(args.steps // 2, 1), 1)
        sweep[f"{kind}{r}"] = {"offsets": kk, "ms": round(mss, 4), "Mlookups_per_s": round(n * kk / mss / 1e3, 1),
                               "hit_rate": round(h, 4)}
    shifted = keys + torch.tensor([1, 0, 0], dtype=torch.int32, device="cuda")
    res = {}

    def inter():
        res["r"] = m.intersect(shifted)
    ims = _timed(inter, max(args.steps // 2, 1), 1)
    sweep["intersect"] = {"ms": round(ims, 4), "Mkeys_per_s": round(n / ims / 1e3, 1), "rows": int(res["r"].shape[0])}
    assert m.device_status() == 0

    # roofline of the lookup kernel: per lookup one random window line, the
    # index and mask outputs, and the query key read once per query
    per_lookup = READ_LINE + 4 + 1 + 12.0 / k
    kern_s = outs["kernel_ms"] / 1e3
    nb_traffic = None
    if (sources_measured() and args.query_order == "given" and args.max_load == 0.5
            and (args.neighbors_probe_group, args.neighbors_bucket_width) == (1, 4)):
        nb_traffic = round(MEASURED_TRAFFIC_NEIGHBORS / 1e9, 2)
    achieved = per_lookup * n * k / kern_s / 1e9
    cpu = None
    if args.cpu_sample > 0:
        from oracle import OracleMap
        s = min(max(args.cpu_sample // 10, 1), n)
        om = OracleMap(n, 3)
        om.insert(keys_np)
        off_np = ash.neighbor_offsets("radius", 1, device=None).numpy()
        c0 = time.perf_counter()
        om.find_offsets(keys_np[:s], off_np)
        c1 = time.perf_counter()
        cpu = {"value": round(s * k / (c1 - c0) / 1e6, 3), "unit": "Mlookups/s", "cores": 1, "kind": "oracle",
               "sample": f"27-neighborhoods of the first {s} cells ({c1 - c0:.1f} s; map of all {n} cells built untimed)"}
    print(json.dumps({
        "metric": "Mlookups/s neighbor search (27 radius-1 neighbors of every cell)",
        "value": round(n * k / ms / 1e3, 1), "unit": "Mlookups/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{n} distinct 5 mm lattice cells of 5M surface points; queries = the cells",
                   "query_order": args.query_order, "probe_group": args.neighbors_probe_group,
                   "bucket_width": args.neighbors_bucket_width, "max_load": args.max_load, "sweep": sweep},
        "roofline": {"bound": "hbm", "kernel": "find_offsets", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": nb_traffic,
                     "traffic_unit": "GB per launch",
                     "algorithmic_bytes_per_lookup": round(per_lookup, 2), "kernel_ms": round(outs["kernel_ms"], 4)},
        "cpu_baseline": cpu}), flush=True)


class ServedWorkload:
    """The served map's workload: capacity 2^25, 20M keys preloaded with
    f32x8 rows, and a Poisson stream of requests (60% find, 30% insert, 10%
    erase; sizes log-uniform in [256, 2^20]; keys uniform over the 318^3 key
    universe, taken as slices of device-resident key pools) replayed through
    the continuous-batching server.  Offered load sets the mean arrival rate
    in key operations per second."""

    def __init__(self, args, n_requests):
        import torch

        import paper_2110_00511_amd as ash
        import synth
        from paper_2110_00511_amd import _lib as L

        self.ash, self.args = ash, args
        w = synth.served(n_requests=n_requests)
        self.w = w
        self.m = ash.HashMap(w["capacity"], 3, [(torch.float32, 8)], max_load=args.served_max_load,
                             probe_group=args.served_probe_group, bucket_width=args.served_bucket_width)
        self.m.insert(torch.from_numpy(w["preload_keys"]).cuda(), [torch.from_numpy(w["preload_values"]).cuda()])
        torch.cuda.synchronize()
        pool = 1 << 24
        g = torch.Generator(device="cuda").manual_seed(w["seed"])
        self.kpool = torch.randint(0, w["side"], (pool + (1 << 20), 3), dtype=torch.int32, device="cuda", generator=g)
        self.vpool = torch.randn((pool + (1 << 20), 8), dtype=torch.float32, device="cuda", generator=g)
        opool = 1 << 25
        self.oidx = torch.empty(opool + (1 << 20), dtype=torch.int32, device="cuda")
        self.omask = torch.empty(opool + (1 << 20), dtype=torch.uint8, device="cuda")
        rng = np.random.default_rng(w["seed"] + 1)
        kinds, sizes = w["kinds"], w["sizes"]
        offs = rng.integers(0, pool, size=len(kinds))
        self.vptrs, self.reqs = [], []
        out_off = 0
        for k, n, o in zip(kinds, sizes, offs):
            o, n = int(o), int(n)
            vp = None
            if k == 1:
                arr = (ctypes.c_void_p * 1)(self.vpool[o].data_ptr())
                self.vptrs.append(arr)
                vp = ctypes.cast(arr, ctypes.c_void_p)
            self.reqs.append(L.AshRequest(int(k), self.kpool[o].data_ptr(), n, vp,
                                          self.oidx[out_off].data_ptr() if k != 2 else None,
                                          self.omask[out_off].data_ptr(), None))
            out_off = (out_off + n) % opool
        self.sizes = sizes
        self.mean_ops = float(sizes.sum()) / len(sizes)

    def run(self, load_ops_per_s, fuse, count):
        """Replays the first `count` requests (None load: all arriving at once)."""
        srv = self.ash.Server(self.m, fuse=fuse, in_flight=self.args.served_in_flight,
                              max_batch=self.args.served_max_batch)
        gaps = self.w["gaps"][:count] * (self.mean_ops / load_ops_per_s) if load_ops_per_s else np.zeros(count)
        lat, sts, span = srv.replay(self.reqs[:count], np.cumsum(gaps) - gaps[0])
        st = srv.stats()
        srv.close()
        ops = int(self.sizes[:count].sum())
        return dict(ops_per_s=ops / span, p50_ms=float(np.percentile(lat, 50) * 1e3),
                    p99_ms=float(np.percentile(lat, 99) * 1e3), span_s=span, batches=st["batches"],
                    largest_batch_requests=st["largest"], requests=count, ops=ops, failed=int((sts != 0).sum()))

    def run_plain(self, count):
        """The plain single-map path on the same stream: the first `count`
        requests as direct ash_insert / ash_find / ash_erase calls on one
        stream, one after another in arrival order, no server; returns the
        throughput from the first call to the end of the last one."""
        import torch

        from paper_2110_00511_amd import _lib as L
        lib = L.load()
        sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        m = self.m._m
        calls = {0: lambda r: lib.ash_find(m, r.keys, r.n, r.out_idx, r.out_mask, None, sp),
                 1: lambda r: lib.ash_insert(m, r.keys, r.n, r.values, r.out_idx, r.out_mask, sp),
                 2: lambda r: lib.ash_erase(m, r.keys, r.n, r.out_mask, sp)}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in self.reqs[:count]:
            L.check(calls[r.kind](r), "plain-path request")
        torch.cuda.synchronize()
        span = time.perf_counter() - t0
        ops = int(self.sizes[:count].sum())
        return dict(ops_per_s=ops / span, span_s=span, requests=count, ops=ops)

    def close(self):
        self.m.close()


def _rounded(d):
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}


def served_leg(args):
    """The served map beside the plain path on the same request stream: the
    plain path's mixed throughput (every request a direct call, one after
    another on one stream), the server's burst capacity (every request
    waiting), then the stream offered at 0.5x and 0.9x of the plain path's
    mixed throughput, fused and one request per batch."""
    work = ServedWorkload(args, args.requests)
    try:
        plain = work.run_plain(len(work.reqs))
        basis = plain["ops_per_s"]
        cal = work.run(None, True, min(len(work.reqs), 5000))
        out = {"plain_path_mixed_Mops": round(basis / 1e6, 1), "offered_load_basis": "plain_path_mixed_Mops",
               "burst_capacity_Mops": round(cal["ops_per_s"] / 1e6, 1)}
        for load in (0.5, 0.9):
            for fuse in (True, False):
                r = work.run(load * basis, fuse, len(work.reqs))
                out[f"{'fused' if fuse else 'unfused'}_{load}x"] = _rounded(
                    {"Mops": r["ops_per_s"] / 1e6, "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
                     "span_s": r["span_s"], "batches": r["batches"], "largest_batch_requests":
                     r["largest_batch_requests"], "failed": r["failed"]})
        out["workload"] = (f"capacity 2^25, 20M preloaded int32x3 keys with f32x8 rows, {len(work.reqs)} Poisson "
                           "requests (60% find / 30% insert / 10% erase, sizes log-uniform in [256, 2^20]); "
                           "latency = completion - scheduled arrival")
        out["server"] = {"max_load": args.served_max_load, "probe_group": args.served_probe_group,
                         "bucket_width": args.served_bucket_width, "in_flight": args.served_in_flight,
                         "max_batch": args.served_max_batch, "max_fused": 256}
        return out
    finally:
        work.close()


def bench_served(args):
    """Served map on its own: burst capacity, then the stream at 0.5x and
    0.9x of the plain path's mixed throughput on the same stream (or of
    --served-basis-mops), fused and one request per batch."""
    import torch
    torch.cuda.set_device(0)
    work = ServedWorkload(args, args.requests)
    cal = work.run(None, True, min(len(work.reqs), 5000))  # burst: everything waiting, the server's capacity
    cap = cal["ops_per_s"]
    if args.served_burst_only:
        print(json.dumps({"metric": "served map burst capacity (every request waiting)",
                          "value": round(cap / 1e6, 1), "unit": "Mops/s", "n_gpus": 1, "higher_is_better": True,
                          "dtype": "int32", "data": "synthetic", "burst": _rounded(cal)}), flush=True)
        work.close()
        return
    plain = None
    if args.served_basis_mops:
        basis = args.served_basis_mops * 1e6
    else:
        plain = work.run_plain(len(work.reqs))
        basis = plain["ops_per_s"]
    out = {}
    for load in (0.5, 0.9):
        out[f"fused_{load}"] = work.run(load * basis, True, len(work.reqs))
        out[f"unfused_{load}"] = work.run(load * basis, False, len(work.reqs))
    head = out["fused_0.9"]
    print(json.dumps({
        "metric": "served map ops/s with p50/p99 latency (continuous batching)",
        "value": round(head["ops_per_s"] / 1e6, 1), "unit": "Mops/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": "int32", "data": "synthetic",
        "p50_ms": round(head["p50_ms"], 3), "p99_ms": round(head["p99_ms"], 3),
        "config": {"workload": f"capacity 2^25, 20M preloaded keys, f32x8 values, {len(work.reqs)} Poisson requests "
                               "(60% find / 30% insert / 10% erase, sizes log-uniform in [256, 2^20])",
                   "burst_capacity_Mops": round(cap / 1e6, 1), "offered_load_basis_Mops": round(basis / 1e6, 1),
                   "offered_load_basis": "given" if plain is None else "plain path, same stream, back to back",
                   "mean_request_ops": round(work.mean_ops),
                   "max_load": args.served_max_load, "probe_group": args.served_probe_group,
                   "bucket_width": args.served_bucket_width, "in_flight": args.served_in_flight,
                   "max_batch": args.served_max_batch},
        "runs": {k: _rounded(v) for k, v in out.items()}}), flush=True)
    work.close()


if __name__ == "__main__":
    main()
