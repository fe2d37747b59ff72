// Continuous-batching server: independent runs of different mesh and particle
// sizes share one GPU.  An admission thread takes jobs in arrival order when
// their device footprint fits the HBM budget and a slot is free; each
// admitted run is driven by a slot thread on its own HIP stream, so steps of
// resident runs overlap on the device; a finished run frees its memory and
// its slot for the next job.  Every run is self-contained (no state is shared
// between runs), so a result is identical alone and in the mix.
#include <hip/hip_runtime_api.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fempic_impl.h"
#include "run.h"

using namespace fempic;
using clk = std::chrono::steady_clock;

namespace {

struct Job {
    int64_t ticket = 0;
    fempic_job spec{};
    std::vector<double> pos, vel;
    size_t footprint = 0;
    clk::time_point t_submit, t_admit, t_done;
    int32_t status = FEMPIC_EAGAIN;
    bool done = false;
    std::vector<double> e, b, rpos, rvel, step_ms;
    std::string message;  // why it failed
    double gauss[3] = {0, 0, 0};
};

// the same estimate as fempic_footprint for the N^3 Kuhn cube
size_t cube_footprint(int N, int order, int64_t n, bool mixed, bool absorbing)
{
    FootprintSizes z = kuhn_sizes(order, 6.0 * N * N * N);
    z.absorbing = absorbing;
    return footprint_bytes(z, n, mixed);
}

}  // namespace

struct fempic_server_s {
    fempic_server_params prm{};
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Job>> queue;
    std::map<int64_t, std::shared_ptr<Job>> jobs;
    // slot threads with their jobs; a finished one is joined the next time the
    // admission thread wakes (its job is done, so it no longer needs the lock)
    std::vector<std::pair<std::thread, std::shared_ptr<Job>>> slots;
    std::thread admit;
    int64_t next_ticket = 1;
    size_t used = 0;
    int resident = 0;
    bool stop = false;
    int device = 0;

    void slot_main(std::shared_ptr<Job> j)
    {
        (void)hipSetDevice(device);
        int32_t st = FEMPIC_OK;
        std::string msg;
        try {
            std::shared_ptr<const HostMesh> mesh(build_cube(j->spec.N, j->spec.L, j->spec.order));
            // the run may not grow past what the job was admitted with
            Run run(mesh, j->spec.params, nullptr, j->footprint);
            // small runs are launch-bound: their particle phases replay graphs
            run.set_phase_graphs(true);
            run.load(j->pos.data(), j->vel.data(), j->spec.n, j->spec.q, j->spec.m, j->spec.w);
            for (int s = 0; s < j->spec.n_steps; s++) {
                run.step(1);
                j->step_ms.push_back(std::chrono::duration<double, std::milli>(clk::now() - j->t_admit).count());
            }
            run.gauss(j->gauss);
            j->e.resize(mesh->N1);
            j->b.resize(mesh->N2);
            run.fields_get(j->e.data(), mesh->N1, j->b.data(), mesh->N2);
            j->rpos.resize(3 * j->spec.n);
            j->rvel.resize(3 * j->spec.n);
            run.particles_get(j->rpos.data(), j->rvel.data(), nullptr, j->spec.n);
        } catch (const Error &e) {
            st = e.code;
            msg = e.what();
        } catch (...) {
            st = FEMPIC_EDEVICE;
            msg = "unknown failure";
        }
        std::lock_guard<std::mutex> lk(mu);
        j->status = st;
        j->message = msg;
        j->t_done = clk::now();
        j->done = true;
        j->pos.clear();
        j->pos.shrink_to_fit();
        j->vel.clear();
        j->vel.shrink_to_fit();
        used -= j->footprint;
        resident--;
        cv.notify_all();
    }

    // join the slot threads whose jobs are done (called with mu held)
    void reap()
    {
        for (size_t k = 0; k < slots.size();) {
            if (slots[k].second->done) {
                slots[k].first.join();
                slots[k] = std::move(slots.back());
                slots.pop_back();
            } else {
                k++;
            }
        }
    }

    void admit_main()
    {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            cv.wait(lk, [&] {
                if (stop) return true;
                reap();
                if (queue.empty()) return false;
                auto &j = queue.front();
                return resident < prm.max_slots && used + j->footprint <= prm.hbm_budget;
            });
            if (stop) break;
            reap();
            auto j = queue.front();
            queue.pop_front();
            used += j->footprint;
            resident++;
            j->t_admit = clk::now();
            slots.emplace_back(std::thread(&fempic_server_s::slot_main, this, j), j);
        }
    }
};

#define API_TRY try {
#define API_CATCH                               \
    }                                           \
    catch (const Error &e) {                    \
        set_error(e.what());                    \
        return e.code;                          \
    }                                           \
    catch (const std::exception &e) {          \
        set_error(e.what());                    \
        return FEMPIC_EINVAL;                   \
    }

extern "C" {

int32_t fempic_server_create(const fempic_server_params *params, fempic_server *out)
{
    API_TRY
    if (!params || !out || params->max_slots < 1 || params->hbm_budget == 0) throw Error(FEMPIC_EINVAL, "bad server parameters");
    auto *s = new fempic_server_s();
    s->prm = *params;
    (void)hipGetDevice(&s->device);
    s->admit = std::thread(&fempic_server_s::admit_main, s);
    *out = s;
    return FEMPIC_OK;
    API_CATCH
}

int32_t fempic_server_destroy(fempic_server s)
{
    if (!s) return FEMPIC_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    s->admit.join();
    for (auto &t : s->slots) t.first.join();
    delete s;
    return FEMPIC_OK;
}

int32_t fempic_submit(fempic_server s, const fempic_job *job, int64_t *ticket)
{
    API_TRY
    if (!s || !job || !ticket) throw Error(FEMPIC_EINVAL, "null argument");
    if (job->N < 1 || job->N > CUBE_N_MAX || (job->order != 1 && job->order != 2) || job->n < 0 || job->n_steps < 0 ||
        (job->n > 0 && (!job->pos || !job->vel)))
        throw Error(FEMPIC_EINVAL, "bad job");
    check_params(job->params);
    auto j = std::make_shared<Job>();
    j->spec = *job;
    j->pos.assign(job->pos, job->pos + 3 * job->n);
    j->vel.assign(job->vel, job->vel + 3 * job->n);
    j->spec.pos = nullptr;
    j->spec.vel = nullptr;
    j->footprint = cube_footprint(job->N, job->order, job->n, job->params.precision == FEMPIC_MIXED,
                                  job->params.field_bc == FEMPIC_FIELD_ABSORB);
    if (j->footprint > s->prm.hbm_budget) throw Error(FEMPIC_ENOMEM, "job can never fit the HBM budget");
    j->t_submit = clk::now();
    std::lock_guard<std::mutex> lk(s->mu);
    j->ticket = s->next_ticket++;
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    s->cv.notify_all();
    *ticket = j->ticket;
    return FEMPIC_OK;
    API_CATCH
}

int32_t fempic_poll(fempic_server s, int64_t ticket, fempic_job_result *out)
{
    API_TRY
    if (!s || !out) throw Error(FEMPIC_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) throw Error(FEMPIC_EINVAL, "unknown ticket");
    Job &j = *it->second;
    if (!j.done) return FEMPIC_EAGAIN;
    fempic_job_result r{};
    r.status = j.status;
    r.n1 = (int64_t)j.e.size();
    r.n2 = (int64_t)j.b.size();
    r.n = j.spec.n;
    r.e = j.e.data();
    r.b = j.b.data();
    r.pos = j.rpos.data();
    r.vel = j.rvel.data();
    for (int k = 0; k < 3; k++) r.gauss[k] = j.gauss[k];
    r.queue_ms = std::chrono::duration<double, std::milli>(j.t_admit - j.t_submit).count();
    r.run_ms = std::chrono::duration<double, std::milli>(j.t_done - j.t_admit).count();
    r.step_done_ms = j.step_ms.data();
    r.n_steps = (int32_t)j.step_ms.size();
    r.message = j.message.c_str();
    *out = r;
    return FEMPIC_OK;
    API_CATCH
}

int32_t fempic_result_release(fempic_server s, int64_t ticket)
{
    API_TRY
    if (!s) throw Error(FEMPIC_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) throw Error(FEMPIC_EINVAL, "unknown ticket");
    if (!it->second->done) throw Error(FEMPIC_EBUSY, "job still running");
    s->jobs.erase(it);
    return FEMPIC_OK;
    API_CATCH
}

}  // extern "C"
