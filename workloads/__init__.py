"""Seeded synthetic inputs for the augmented-system solver.

This package builds the *inputs* of the solve: the per-time-step Jacobian
blocks of the lifted constraint (N_k, V_k and Z~_k of Sec. 4.1 eq. (blocks)
and Sec. 5.1) on every level of the time hierarchy, and a right-hand side.
It holds none of the solver's arithmetic (no assembly, smoothing, transfer
or Krylov step); both the HIP path and the CPU oracle consume what it makes.

Two model problems are provided, following Sec. 6.1 (van der Pol) and
Sec. 6.2 (viscous Burgers, upwind finite differences, backward Euler).
The linearisation point (the SQP iterate at which the Jacobians are taken)
is random and seeded; it stands in for the iterates of the paper's SQP runs,
which cannot be reproduced.  Every level of the hierarchy is rediscretised
at its own step 2^l * dt, at a linearisation point obtained from the finest
one by injection (states) and averaging (controls), i.e. by the same
restriction the multigrid cycle uses (Sec. 5.3.1).

It also draws the seeded initial parameters of the learned coarse
correction's network (coarse_net_params), and gives the step initial state
of the nonlinear Burgers solve of Sec. 6.2 (burgers_step_state).
"""
from .problems import (Problem, Level, vanderpol_jacobians, burgers_jacobians,
                       lifted_blocks, make_problem, make_rhs, config_problem,
                       coarse_net_params, batch_mix, burgers_step_state, CONFIGS)

__all__ = ["Problem", "Level", "vanderpol_jacobians", "burgers_jacobians",
           "lifted_blocks", "make_problem", "make_rhs", "config_problem",
           "coarse_net_params", "batch_mix", "burgers_step_state", "CONFIGS"]
