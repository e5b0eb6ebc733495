"""Test helper: build and call the host (g++) build of the generated pointwise code."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
GEN = os.path.join(ROOT, "paper_2309_06225_amd", "csrc", "gen")
LIB = os.path.join(HERE, "_host_point.so")
_dp = ctypes.POINTER(ctypes.c_double)
PARAMS = ("lambda_gb", "g2", "kappa1", "kappa3", "k1_1pk2", "k1_2pk2", "k1k2",
          "lapse_coeff", "lapse_advec", "shift_gamma_coeff", "shift_advec", "eta",
          "inv1pa", "a_1pa", "fb", "cfac", "b4", "lambda_lin", "beta")
_lib = None


def lib():
    global _lib
    if _lib is None:
        src = os.path.join(HERE, "host_point.cpp")
        deps = [src] + [os.path.join(GEN, f) for f in ("gen_rhs.inc", "gen_vjp.inc", "gen_layout.h")]
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(d) for d in deps):
            subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-I", GEN, "-o",
                            LIB + ".tmp", src], check=True)
            os.replace(LIB + ".tmp", LIB)
        _lib = ctypes.CDLL(LIB)
    return _lib


def point_params(p: dict) -> np.ndarray:
    a, b, k1, k2 = p["a_gauge"], p["b_gauge"], p["kappa1"], p["kappa2"]
    d = dict(lambda_gb=p["lambda_gb"], g2=p["g2"], kappa1=k1, kappa3=p["kappa3"], k1_1pk2=k1 * (1 + k2),
             k1_2pk2=k1 * (2 + k2), k1k2=k1 * k2, lapse_coeff=p["lapse_coeff"], lapse_advec=p["lapse_advec"],
             shift_gamma_coeff=p["shift_gamma_coeff"], shift_advec=p["shift_advec"], eta=p["eta"],
             inv1pa=1 / (1 + a), a_1pa=a / (1 + a), fb=b / (1 + b), cfac=1 / (1 + b), b4=b / (4 * (1 + b)),
             lambda_lin=p.get("lambda_lin", 0.0), beta=p.get("beta", 0.0))
    return np.array([d[n] for n in PARAMS])


D1_FIELDS = [f for f in range(27) if not (22 <= f < 25)]
D2_FIELDS = [0, 1, 2, 3, 4, 5, 6, 18, 19, 20, 21, 25]


def pack_inputs(d1, d2, advsum):
    """d1[27,3], d2[27,6], advsum[27] -> derivative-buffer vector of 198 components."""
    D = np.zeros(198)
    for s, f in enumerate(D1_FIELDS):
        D[3 * s:3 * s + 3] = d1[f]
    for s, f in enumerate(D2_FIELDS):
        D[72 + 6 * s:72 + 6 * s + 6] = d2[f]
    D[144:171] = advsum
    return D


def rhs_point(pp, u, D, sa=1):
    out = np.zeros(27)
    bad = lib().host_rhs_point(int(sa), pp.ctypes.data_as(_dp), np.ascontiguousarray(u).ctypes.data_as(_dp),
                               np.ascontiguousarray(D).ctypes.data_as(_dp), out.ctypes.data_as(_dp))
    return out, bad


def vjp_point(pp, u, D, w, sa=1):
    ub, Db, tb = np.zeros(27), np.zeros(198), np.zeros(2)
    lib().host_vjp_point(int(sa), pp.ctypes.data_as(_dp), np.ascontiguousarray(u).ctypes.data_as(_dp),
                         np.ascontiguousarray(D).ctypes.data_as(_dp), np.ascontiguousarray(w).ctypes.data_as(_dp),
                         ub.ctypes.data_as(_dp), Db.ctypes.data_as(_dp), tb.ctypes.data_as(_dp))
    return ub, Db, tb
