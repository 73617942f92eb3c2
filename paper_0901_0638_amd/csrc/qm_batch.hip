/* qm_batch.hip -- persistent batch kernel (placeholder). */
