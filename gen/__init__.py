"""Seeded synthetic electron-event inputs (shared by tests and the benchmark)."""
from .synth import (WORKLOADS, C4_TRUE_ABERRATIONS, LAMBDA_300KV, EventData, Workload, simulate,
                    random_csr, with_pileup, shuffle_within_frames, probe_spectrum, run_length_form)

__all__ = ["WORKLOADS", "C4_TRUE_ABERRATIONS", "LAMBDA_300KV", "EventData", "Workload", "simulate",
           "random_csr", "with_pileup", "shuffle_within_frames", "probe_spectrum",
           "run_length_form"]
