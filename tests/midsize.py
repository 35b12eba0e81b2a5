"""Workloads of the small workload's shape on the rings between the small ring and the
benchmark's (N = 2^13 .. 2^15, 12 + alpha primes), registered by name on first use."""
import synth


def mid_workload(log_n, alpha):
    """the name of the workload on a 2^log_n ring with 12 + alpha primes, three CoeffToSlot
    groups and as many conv channels as the ring's slots hold (C = N / 32^2, 16 x 16 image)"""
    name = "mid%d_a%d" % (log_n, alpha)
    if name not in synth.WORKLOADS:
        w = dict(synth.WORKLOADS["small"])
        C = (1 << log_n) // 1024
        w.update({"description": "N = 2^%d, 12 + %d primes, 3x3 conv %d->%d on 16x16, CoeffToSlot in 3 groups"
                                 % (log_n, alpha, C, C),
                  "log_n": log_n, "n_q": 12, "alpha": alpha, "cts_groups": 3, "c_in": C, "c_out": C,
                  "data_seed": 1100 + log_n, "key_seed": 2100 + log_n + 20 * alpha})
        synth.WORKLOADS[name] = w
    return name
