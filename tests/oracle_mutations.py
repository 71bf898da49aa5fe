"""Mutation check of the oracle's pins (test infrastructure, not collected by pytest).

Each mutation is one plausible slip in the oracle (a dropped factor, a flipped
sign, a wrong index or node, a branch taken the other way), applied alone to a
scratch copy of oracle/hwe_oracle.cpp under /tmp; the copy is compiled and the
CPU oracle tests are run against it.  A mutation must make at least one of
them fail.  The operation-count test (its constants follow any change of the
arithmetic) and the round-off growth tests (they measure sensitivity, not
correctness) are left out, so that a catch is made by a pin.

usage: python tests/oracle_mutations.py [name ...]      (all mutations by default)
"""
import os
import shutil
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NOT_PINS = "not flop_constants and not amplifies_round_off"

MUT = [
 ("kappa_ninth", "T kappa = tsum * tsum / T(9.0);", "T kappa = tsum * tsum;"),
 ("wave_quarter", "/ T(4.0) + T(1e-30)", "/ T(3.0) + T(1e-30)"),
 ("alpha_max", "alpha = k < F.nb ? maxfirst(aK, aN) : maxfirst(aN, aK);", "alpha = val(aK) < val(aN) ? aK : aN;"),
 ("dt_inradius", "rmin = std::min(rmin, 2.0 * M->area[k] / per);", "rmin = std::min(rmin, M->area[k] / per);"),
 ("beta0_area2", "b += T(A0 * A0) * (dxx * dxx", "b += T(A0) * (dxx * dxx"),
 ("beta0_dxx", "T dxx = T(2.0) * a[3], dxy = a[4], dyy = T(2.0) * a[5];", "T dxx = a[3], dxy = a[4], dyy = a[5];"),
 ("beta_area", "T b = T(A0) * (dx * dx + dy * dy);", "T b = (dx * dx + dy * dy);"),
 ("omega_frac2", "wb[l] = T(o.lin_w[l]) * (T(1.0) + frac);", "wb[l] = T(o.lin_w[l]) * (T(1.0) + T(2.0) * frac);"),
 ("D_eps_power", "T D = w2 * w2 * T(o.eps) + w2 * beta[l];", "T D = w2 * T(o.eps) + w2 * beta[l];"),
 ("D_beta_scale", "T D = w2 * w2 * T(o.eps) + w2 * beta[l];", "T D = w2 * w2 * T(o.eps) + beta[l];"),
 ("recon_sign", "inner -= T(o.lin_w[l] / g1) * pv[l][j];", "inner += T(o.lin_w[l] / g1) * pv[l][j];"),
 ("recon_g1", "T inner = pv[0][j] / T(g1);", "T inner = pv[0][j];"),
 ("eval_dx", "pv[l][1] = a[1] + T(2.0 * X) * a[3] + T(Y) * a[4];", "pv[l][1] = a[1] + T(X) * a[3] + T(Y) * a[4];"),
 ("eval_dyy", "pv[l][5] = T(2.0) * a[5];", "pv[l][5] = a[5];"),
 ("step1_rx3", "rx[3] += w * 2.0 * mxi;", "rx[3] += w * mxi;"),
 ("step1_rhs", "b[(l - 1) * m + q] = (T(st[l].area) * st[l].V[q] + T(A0) * st[0].V[q]) * T(h / A0);",
  "b[(l - 1) * m + q] = (T(st[l].area) * st[l].V[q]) * T(h / A0);"),
 ("step2_index", "b[0 * m + q] = st[l].W[q];", "b[0 * m + q] = st[0].W[q];"),
 ("step2_Y", "b[2 * m + q] = T(wd) * st[l].Y[q];", "b[2 * m + q] = T(wd) * st[l].V[q];"),
 ("taylor_half", "Wi[q] = Di[0][q] + T(tau) * it[q] + T(0.5 * tau * tau) * itt[q];",
  "Wi[q] = Di[0][q] + T(tau) * it[q] + T(tau * tau) * itt[q];"),
 ("taylor_ext", "De[0][q] + T(tau) * et[q] + T(0.5 * tau * tau) * ett[q] : Wi[q];",
  "De[0][q] + T(tau) * it[q] + T(0.5 * tau * tau) * ett[q] : Wi[q];"),
 ("lobatto", "{1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0}", "{1.0 / 4.0, 2.0 / 4.0, 1.0 / 4.0}"),
 ("llf_sign", "T Hhat = T(0.5) * (He + Hi - alpha * (We[q] - Wi[q]));", "T Hhat = T(0.5) * (He + Hi + alpha * (We[q] - Wi[q]));"),
 ("update_sign", "Wn[q] = Wbar[q] - T(dt / A) * Fsum[q];", "Wn[q] = Wbar[q] + T(dt / A) * Fsum[q];"),
 ("gg_normal", "Ys[q] += What * T(F.ny * er.w[G] * F.len);", "Ys[q] += What * T(F.nx * er.w[G] * F.len);"),
 ("interface_time", "taylor(dt, Wi, We);\n        for (int q = 0; q < m; ++q) {\n          T What",
  "taylor(0.5 * dt, Wi, We);\n        for (int q = 0; q < m; ++q) {\n          T What"),
 ("pressure_half", "N p = (o.gas_gamma - 1.0) * (E - 0.5 * (mx * u + my * v));", "N p = (o.gas_gamma - 1.0) * (E - (mx * u + my * v));"),
 ("flux_g2", "g[2] = my * v + p;", "g[2] = my * v;"),
 ("sound_speed", "T c = sqrtv(T(o.gas_gamma) * p / W[0]);", "T c = sqrtv(p / W[0]);"),
 ("reflect_factor", "  W[1] = W[1] - T(2.0 * nx) * mn;\n  W[2] = W[2] - T(2.0 * ny) * mn;\n  T vn",
  "  W[1] = W[1] - T(1.0 * nx) * mn;\n  W[2] = W[2] - T(1.0 * ny) * mn;\n  T vn"),
 ("lw_tx_index", "eval(1, D[1], D[2], D[4], nullptr, a2);", "eval(1, D[1], D[2], D[3], nullptr, a2);"),
 ("lw_tt_sign", "Wtt[q] = T(0.0) - a1[q] - a2[q];", "Wtt[q] = T(0.0) - a1[q] + a2[q];"),
 ("lw_ty_index", "eval(0, D[2], D[1], D[4], nullptr, a1);", "eval(0, D[2], D[1], D[5], nullptr, a1);"),
 ("lim_rho_eps", "R.theta[0] = (Wb[0] - T(eps)) / (Wb[0] - rmin);", "R.theta[0] = (Wb[0]) / (Wb[0] - rmin);"),
 ("lim_b_coef", "T b = T(2.0) * (Ep * dr + Wb[0] * dE) - T(2.0) * (Wb[1] * d1 + Wb[2] * d2);",
  "T b = T(2.0) * (Ep * dr + Wb[0] * dE) - (Wb[1] * d1 + Wb[2] * d2);"),
 ("lim_root_pick", "root = ok1 && ok2 ? (v1 <= v2 ? r1 : r2)", "root = ok1 && ok2 ? (v1 <= v2 ? r2 : r1)"),
 ("rev_div", "return rev_node(q, a.i, 1.0 / b.v, b.i, -q / b.v);", "return rev_node(q, a.i, 1.0 / b.v, b.i, q / b.v);"),
 ("rev_sqrt", "return rev_node(r, a.i, 0.5 / r, -1, 0.0);", "return rev_node(r, a.i, 1.0 / r, -1, 0.0);"),
 ("dual_div", "return Dual(q, (a.d - q * b.d) / b.v);", "return Dual(q, (a.d + q * b.d) / b.v);"),
 ("dual_abs", "inline Dual absval(Dual a) { return Dual(std::fabs(a.v), sgn0(a.v) * a.d); }",
  "inline Dual absval(Dual a) { return Dual(std::fabs(a.v), a.d); }"),

 ("edge3_weights", "{5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0}", "{1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0}"),
 ("edge3_nodes", "{0.5 - 0.38729833462074168852, 0.5, 0.5 + 0.38729833462074168852}", "{0.5 - 0.3, 0.5, 0.5 + 0.3}"),
 ("gl_time_nodes", "{2, {0.5 - 0.28867513459481288225, 0.5 + 0.28867513459481288225, 0.0},\n                                 {0.5, 0.5, 0.0}}",
  "{2, {0.25, 0.75, 0.0},\n                                 {0.5, 0.5, 0.0}}"),
 ("moving_tbnd_run", "M->t_bnd = M->time + (double(n) + 0.5) * dt;", "M->t_bnd = M->time + (double(n) + 1.0) * dt;"),
 ("prescribed_ext", "if (F.nb < 0 && prescribed(F)) boundary_state(M, F, We);", "if (false) boundary_state(M, F, We);"),
 ("prescribed_ghost_flat", "for (int q = 0; q < m; ++q) c.V[q] = c.Y[q] = T(0.0);", ";"),
 ("ghost_V_mirror", "c.V[q] = st[0].V[q] - T(2.0 * F.nx) * vn;", "c.V[q] = st[0].V[q];"),
 ("periodic_shift", "eval_recon(o, R[F.nb], q, xg - F.sx, yg - F.sy, tmp);", "eval_recon(o, R[F.nb], q, xg + F.sx, yg + F.sy, tmp);"),
 ("ghost_geom_shift", "c.t.x[v] += F.sx;", "c.t.x[v] -= F.sx;"),
 ("burgers_sr", "if (o.eq == 1) return absval(W[0] * T(nx + ny));", "if (o.eq == 1) return absval(W[0]) * T(nx + ny);"),
 ("adv_sr", "if (o.eq == 0) return T(std::fabs(o.adv[0] * nx + o.adv[1] * ny));",
  "if (o.eq == 0) return T(std::fabs(o.adv[0] * nx) + std::fabs(o.adv[1] * ny));"),
 ("limiter_eval", "D[0] = R.wbar[q] + R.theta[q] * (D[0] - R.wbar[q]);", "D[0] = R.theta[q] * D[0];"),
 ("gg_area", "Vn[q] = Vs[q] / T(A);", "Vn[q] = Vs[q] / T(2.0 * A);"),
 ("step2_wd", "double A[9] = {1.0, avg_x(st[l].t), avg_y(st[l].t), 0.0, wd, 0.0, 0.0, 0.0, wd};",
  "double A[9] = {1.0, avg_x(st[l].t), avg_y(st[l].t), 0.0, 1.0, 0.0, 0.0, 0.0, wd};"),
 ("recon_w0", "T r = w[0] * inner;", "T r = w[0] * pv[0][j];"),
 ("moving_tbnd_step", "M->t_bnd = M->time + 0.5 * dt;", "M->t_bnd = M->time + dt;"),
]
# lim_root_pick is an equivalent mutation: the scaling's quadratic is positive
# at 0 and negative at 1, so it has exactly one root in [0, 1] and the branch
# that chooses between two is not reached; it is listed to record that.
EQUIVALENT = {"lim_root_pick"}


def main(names):
    dst = tempfile.mkdtemp(prefix="oracle_mut_")
    try:
        for d in ("oracle", "tests", "workloads"):
            shutil.copytree(os.path.join(ROOT, d), os.path.join(dst, d),
                            ignore=shutil.ignore_patterns("__pycache__", "*.so"))
        shutil.copy(os.path.join(ROOT, "pytest.ini"), dst)
        src = os.path.join(ROOT, "oracle", "hwe_oracle.cpp")
        orig = open(src).read()
        survived = []
        for name, old, new in MUT:
            if names and name not in names:
                continue
            if old not in orig:
                print(f"{name}: pattern not found", flush=True)
                survived.append(name)
                continue
            open(os.path.join(dst, "oracle", "hwe_oracle.cpp"), "w").write(orig.replace(old, new, 1))
            lib = os.path.join(dst, "oracle", "libhwe_oracle.so")
            r = subprocess.run(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", lib,
                                os.path.join(dst, "oracle", "hwe_oracle.cpp")], capture_output=True, text=True)
            if r.returncode:
                print(f"{name}: does not compile", flush=True)
                survived.append(name)
                continue
            t0 = time.time()
            r = subprocess.run([sys.executable, "-m", "pytest", "tests", "-q", "-x", "-m", "not gpu", "-n", "6",
                                "-k", f"oracle and {NOT_PINS}"], cwd=dst, capture_output=True, text=True)
            failed = [l.split(" ")[1] for l in r.stdout.splitlines() if l.startswith("FAILED")]
            if r.returncode and failed:
                print(f"{name}: caught by {failed[0]} ({time.time() - t0:.0f} s)", flush=True)
            else:
                tag = "equivalent, not caught" if name in EQUIVALENT else "NOT CAUGHT"
                print(f"{name}: {tag} ({time.time() - t0:.0f} s)", flush=True)
                if name not in EQUIVALENT:
                    survived.append(name)
        return 1 if survived else 0
    finally:
        shutil.rmtree(dst, ignore_errors=True)


if __name__ == "__main__":
    sys.exit(main(set(sys.argv[1:])))
