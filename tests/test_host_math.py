"""Host-side helpers of the C ABI (no device work): the camera-IMU twist map
and the IESKF pose update, against the oracle's plain forms of Appendix A."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2501_08672_amd import _abi as A
from paper_2501_08672_amd import ops


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_imu_to_camera_twist_matches_oracle(oracle, seed):
    rng = np.random.default_rng(seed)
    R_CI = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    t_CI = rng.normal(0, 0.3, 3)
    R_CW = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    np.testing.assert_allclose(ops.imu_to_camera_twist(R_CI, t_CI, R_CW), oracle.imu_to_camera_twist(R_CI, t_CI, R_CW),
                               rtol=0, atol=1e-14)


@pytest.mark.parametrize("with_prior_offset", [False, True])
def test_ieskf_pose_update_matches_oracle(oracle, with_prior_offset):
    rng = np.random.default_rng(7)
    H = rng.normal(size=(50, 6))
    Rinv = rng.uniform(0.5, 2.0, 50)
    z = rng.normal(size=50)
    L = rng.normal(size=(6, 6))
    P = L @ L.T + 0.1 * np.eye(6)
    dx = rng.normal(0, 0.05, 6) if with_prior_offset else None
    HtRH, HtRz = H.T @ (Rinv[:, None] * H), H.T @ (Rinv * z)
    d_gpu, P_gpu = ops.ieskf_pose_update(HtRH, HtRz, P, dx)
    d_orc, P_orc = oracle.ieskf_pose_update(HtRH, HtRz, P, dx)
    np.testing.assert_allclose(d_gpu, d_orc, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(P_gpu, P_orc, rtol=1e-10, atol=1e-13)


def test_ieskf_pose_update_rejects_singular_prior():
    with pytest.raises(A.GslError) as e:
        ops.ieskf_pose_update(np.eye(6), np.zeros(6), np.zeros((6, 6)))
    assert e.value.code == A.GSL_EINVAL
    assert A.lib().gsl_ieskf_pose_update(None, None, None, None, None, None) == A.GSL_EINVAL
    assert A.lib().gsl_imu_to_camera_twist(None, None, None, None) == A.GSL_EINVAL
    assert "NULL" in A.lib().gsl_last_error().decode()


@pytest.mark.parametrize("noise_var,with_prior_offset", [(1.0, False), (0.04, True)])
def test_ieskf_visual_update_matches_oracle(oracle, noise_var, with_prior_offset):
    """gsl_ieskf_visual_update (H_imu = H_cam A, Appendix A) against the
    oracle's camera-to-IMU chain and update."""
    rng = np.random.default_rng(8)
    H = rng.normal(size=(80, 6))
    z = rng.normal(size=80)
    R_CI = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    t_CI = rng.normal(0, 0.3, 3)
    R_CW = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    A_imu = oracle.imu_to_camera_twist(R_CI, t_CI, R_CW)
    L = rng.normal(size=(6, 6))
    P = L @ L.T + 0.1 * np.eye(6)
    dx = rng.normal(0, 0.05, 6) if with_prior_offset else None
    d_gpu, P_gpu = ops.ieskf_visual_update(H.T @ H, H.T @ z, A_imu, P, dx, noise_var=noise_var)
    d_orc, P_orc = oracle.ieskf_visual_update(H.T @ H, H.T @ z, A_imu, P, dx, noise_var=noise_var)
    np.testing.assert_allclose(d_gpu, d_orc, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(P_gpu, P_orc, rtol=1e-10, atol=1e-13)


def test_ieskf_visual_update_rejects_bad_noise():
    for nv in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(A.GslError) as e:
            ops.ieskf_visual_update(np.eye(6), np.zeros(6), np.eye(6), np.eye(6), noise_var=nv)
        assert e.value.code == A.GSL_EINVAL
