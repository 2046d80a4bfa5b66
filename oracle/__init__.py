"""CPU FP64 oracle for the demag + exchange + LLG hot path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and its
Python binding) imports, links or executes this package; only the tests, the
smoke check and the CPU-baseline leg of the benchmark do. It shares no code,
header, table or constant generator with the HIP path.

What it computes, in plain and slow form:

* ``tensor``  -- the cell-averaged demag tensor N(r) (Newell's f/g functions with
  the 27-point stencil, binary128, inside a switch radius; a moment-matched
  dipole quadrature outside), its periodic wrap and its (real) spectrum.
* ``field``   -- the demag field H = -N (*) (Ms m) as a zero-padded FFT
  convolution (numpy's FFT as the library step), as an O(N^2) direct sum, and a
  naive DFT; the 6-point exchange field; the DMI, uniaxial anisotropy and
  Slonczewski spin-transfer fields; the FP64 energies.
* ``llg``     -- the LLG right-hand side, the classic RK4 step and the RKF45
  step with its step-size control.
* ``adjoint`` -- vector-Jacobian products of h_eff and of one RK4 step.
* ``minimize`` -- energy minimisation with Barzilai-Borwein step sizes.

Parity status per function is stated in each module's docstring.
"""
from .tensor import (tensor_octant, tensor_at, newell_at, far_at, newell_scale_at,
                     wrap_full, tensor_spectrum, default_L, is_7smooth)
from .field import (MU0, HBAR, E_CHARGE, demag_fft, demag_direct, demag_direct_at, naive_dft, exchange_field, exchange_at,
                    dmi_field, anisotropy_field, stt_field, h_eff, energies)
from .llg import (llg_rhs, rk4_step, rk4_run, macrospin_closed_form, rkf45_step, rkf45_run, rkf45_stages,
                  RKF45_A, RKF45_B4, RKF45_B5, RKF45_C)
from .adjoint import h_eff_vjp, llg_rhs_vjp, rk4_step_vjp, rk4_run_grad_Ms
from .minimize import bb_minimize, torque_dir, total_energy
